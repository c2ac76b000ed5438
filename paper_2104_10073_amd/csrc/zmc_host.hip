// zmc_host.hip -- host runtime of the C ABI in include/zmc.h.
//
// Responsibilities: validate and pack function tables (FP64 coefficients in the
// reference operation order, FP32 local-coordinate coefficients derived in FP64
// and rounded once), admit requests into device function slots and a tile-
// partial arena as space frees up, cut functions into tiles, order tiles by
// cost, and enqueue launches (persistent FP32 kernel, persistent FP64 kernel,
// finalize, result copy) on the caller's stream from a small ring of launch
// slots, each with a captured HIP graph -- or, in a resident context, feed one
// persistent kernel through a ring in pinned memory.  Also: promotion of FP32
// results to FP64, run-time compiled families, parameter grids, abort and
// cancellation, checkpoint and resume, tuning, the plain comparator paths.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <sched.h>
#include <time.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/zmc.h"
#include "zmc_device.hpp"
#include "zmc_pack.hpp"

namespace zmc {
const void* plain_kernel_ptr();
const void* batched_kernel_ptr(bool fp64);
const void* finalize_kernel_ptr();
const void* stage_kernel_ptr();
const void* publish_kernel_ptr();
const void* pack_grid_kernel_ptr();
const void* pack_table_kernel_ptr();
const void* sample_points_kernel_ptr();
const void* plain_reduce_kernel_ptr();
const void* resident_kernel_ptr();
// Texts of zmc_device.hpp and zmc_device_code.hpp (generated at build time) for
// compiling caller-supplied families at run time.
extern const char* const kRtcHeaderDevice;
extern const char* const kRtcHeaderCode;
}  // namespace zmc

using namespace zmc;

// Device memory of mc_integrate_plain_fp64_noalloc, for callers that cannot
// allocate: a fixed array in the library's code object, one copy per GPU,
// held until the process ends.  In host code `scratch` is only a host-side
// stand-in; its address on each GPU is looked up once per device
// (scratch_address, called by mc_create with that device current) and only
// that address is ever passed to kernels or copies.
constexpr uint64_t kScratchBytes = 24ull << 20;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

static_assert(sizeof(mc_function) == 472, "mc_function layout");
static_assert(sizeof(mc_result) == 48, "mc_result layout");
static_assert(sizeof(mc_config) == 56, "mc_config layout");
static_assert(sizeof(mc_stats) == 88, "mc_stats layout");
static_assert(sizeof(DevResult) == sizeof(mc_result), "result layout");
static_assert(sizeof(Tile) == 16 && sizeof(Fin) == 16 && sizeof(Partial) == 16, "record layout");
static_assert(sizeof(TileRun) == 32 && sizeof(DevFn) % 16 == 0, "staged record layout");

namespace {

thread_local std::string g_thread_error;

// Limits of the no-allocation path (its whole working set lives in `scratch`).
constexpr uint32_t kNoAllocMaxFunctions = 4096;
constexpr uint64_t kNoAllocMaxBlocks = 1ull << 20;  // plain-kernel blocks of one function: N <= 2^30
constexpr uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }
static_assert(align256(kNoAllocMaxFunctions * sizeof(mc_function)) + kNoAllocMaxFunctions * sizeof(DevFn) +
                      align256(kNoAllocMaxFunctions * sizeof(DevResult)) + kNoAllocMaxBlocks * sizeof(Partial) <=
                  kScratchBytes,
              "no-allocation working set");

constexpr int kMaxScratchDevices = 256;
std::mutex g_scratch_mu;
uint8_t* g_scratch_dev[kMaxScratchDevices] = {};

// Device address of `scratch` on device `dev`, which must be current; looked up
// with hipGetSymbolAddress on the first call for that device, then cached.
hipError_t scratch_address(int dev, uint8_t** out)
{
    if (dev < 0 || dev >= kMaxScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (p == nullptr) return hipErrorInvalidSymbol;
        g_scratch_dev[dev] = (uint8_t*)p;
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

constexpr int kLaunchSlots = 3;
constexpr uint64_t kMaxSamples = 1ull << 40;
constexpr uint32_t kTargetTilesPerFn = 1u << 16;

// ---------------------------------------------------------------- small helpers

struct HipError {
    hipError_t e;
    const char* what;
};

// Calls whose failure is not an error of the operation (cleanup, optional
// timing) go through quiet(): HIP keeps the last error of a thread until
// someone reads it, and a stale one would surface in the caller's next HIP call
// (PyTorch checks it after every launch).
inline void quiet(hipError_t e)
{
    if (e != hipSuccess) (void)hipGetLastError();
}

// Failure injection (a testing aid for the error paths): when a context is
// created with MC_FAULT_HIP=n in the environment, the n-th checked HIP call the
// library makes from then on (in any thread) reports failure without being
// made: out of memory for allocations, hipErrorUnknown otherwise.  Each
// mc_create re-arms the countdown from the variable, or disarms it when the
// variable is absent or 0.  Unchecked calls (cleanup, completion polling) are
// never failed.
std::atomic<int64_t> g_fault_countdown{0};

void arm_fault_injection()
{
    const char* v = std::getenv("MC_FAULT_HIP");
    const long long n = v ? std::atoll(v) : 0;
    g_fault_countdown.store(n > 0 ? (int64_t)n : 0, std::memory_order_relaxed);
}

inline bool fault_due()
{
    if (g_fault_countdown.load(std::memory_order_relaxed) <= 0) return false;
    return g_fault_countdown.fetch_sub(1, std::memory_order_relaxed) == 1;
}

inline hipError_t injected_error(const char* what)
{
    return std::strncmp(what, "hipMalloc", 9) == 0 || std::strncmp(what, "hipHostMalloc", 13) == 0
               ? hipErrorOutOfMemory
               : hipErrorUnknown;
}

// Log level (MC_LOG at mc_create): 0 nothing, 1 failures, 2 context-level
// events, 3 every launch and admission.  Lines go to stderr, prefixed "[zmc] ".
std::atomic<int> g_log_level{0};

void arm_log_level()
{
    const char* v = std::getenv("MC_LOG");
    g_log_level.store(v ? std::atoi(v) : 0, std::memory_order_relaxed);
}

inline bool log_on(int level) { return g_log_level.load(std::memory_order_relaxed) >= level; }

__attribute__((format(printf, 2, 3))) void log_msg(int level, const char* fmt, ...)
{
    if (!log_on(level)) return;
    char buf[600];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    std::fprintf(stderr, "[zmc] %s\n", buf);
}

#define HIP_TRY(expr)                                                    \
    do {                                                                 \
        hipError_t e_ = fault_due() ? injected_error(#expr) : (expr);    \
        if (e_ != hipSuccess) throw HipError{e_, #expr};                 \
    } while (0)

// First-fit range allocator over [0, capacity) with coalescing free list.
class RangeAlloc {
public:
    void reset(uint64_t cap)
    {
        cap_ = cap;
        free_.clear();
        if (cap > 0) free_[0] = cap;
        used_ = 0;
    }
    bool alloc(uint64_t n, uint64_t* off)
    {
        if (n == 0) {
            *off = 0;
            return true;
        }
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const uint64_t rest = it->second - n, start = it->first + n;
                free_.erase(it);
                if (rest > 0) free_[start] = rest;
                used_ += n;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t n)
    {
        if (n == 0) return;
        used_ -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint64_t capacity() const { return cap_; }
    uint64_t used() const { return used_; }

private:
    uint64_t cap_ = 0, used_ = 0;
    std::map<uint64_t, uint64_t> free_;
};

// Index of the kernel that evaluates a family at a precision: the two built-in
// kernels, then one FP32/FP64 pair per run-time family.
int kernel_index(uint32_t family, bool f64)
{
    if (family < (uint32_t)kNumFamilies) return f64 ? kKernelBuiltin64 : kKernelBuiltin32;
    return 2 + 2 * (int)(family - kUserFamily0) + (f64 ? 1 : 0);
}

// ---------------------------------------------------------------- validation

// n_user: run-time families registered on the context (ids kUserFamily0 ..
// kUserFamily0 + n_user - 1); 0 where only the built-in families are accepted.
mc_status validate_one(const mc_function& f, uint32_t n_user, std::string* why)
{
    char buf[160];
    const bool user = f.family >= kUserFamily0 && f.family < kUserFamily0 + n_user;
    if (f.family > MC_FAMILY_POLY_PRODUCT && !user) {
        snprintf(buf, sizeof buf, "unsupported family %u", f.family);
        *why = buf;
        return MC_ERR_UNSUPPORTED_FAMILY;
    }
    if (f.dim < 1 || f.dim > MC_MAX_DIM) {
        snprintf(buf, sizeof buf, "dim %u outside 1..%d", f.dim, MC_MAX_DIM);
        *why = buf;
        return MC_ERR_BAD_DIM;
    }
    if (f.n_samples < 2 || f.n_samples > kMaxSamples) {
        snprintf(buf, sizeof buf, "n_samples %llu outside 2..2^40", (unsigned long long)f.n_samples);
        *why = buf;
        return MC_ERR_INVALID_ARG;
    }
    for (uint32_t j = 0; j < f.dim; ++j) {
        if (!std::isfinite(f.lo[j]) || !std::isfinite(f.hi[j]) || !(f.lo[j] < f.hi[j]) ||
            !std::isfinite(f.hi[j] - f.lo[j])) {
            snprintf(buf, sizeof buf, "bounds of coordinate %u are not finite with lo < hi", j);
            *why = buf;
            return MC_ERR_BAD_BOUNDS;
        }
    }
    for (int j = 0; j < MC_N_PARAMS; ++j) {
        if (!std::isfinite(f.params[j])) {
            snprintf(buf, sizeof buf, "params[%d] is not finite", j);
            *why = buf;
            return MC_ERR_BAD_PARAMS;
        }
    }
    if (f.family == MC_FAMILY_GAUSSIAN && !(f.params[1] > 0.0)) {
        *why = "gaussian sigma must be > 0";
        return MC_ERR_BAD_PARAMS;
    }
    if (f.family == MC_FAMILY_POLY_PRODUCT) {
        for (uint32_t j = 0; j < f.dim; ++j) {
            const double d = f.params[MC_PARAM_W0 + j];
            if (!(d >= 0.0 && d <= (double)kMaxPolyDegree && d == std::floor(d))) {
                snprintf(buf, sizeof buf, "polynomial degree of coordinate %u must be an integer in 0..%d", j,
                         kMaxPolyDegree);
                *why = buf;
                return MC_ERR_BAD_PARAMS;
            }
        }
    }
    return MC_OK;
}

// ---------------------------------------------------------------- packing
// (zmc::pack_function, shared with the grid kernel: zmc_pack.hpp)

// Relative VALU cost of one sample (full-rate issue slots), used to order tiles.
double sample_cost(uint32_t family, uint32_t dim, int precision)
{
    const double philox = 15.0 * dim;
    double fam;
    switch (family) {
    case MC_FAMILY_HARMONIC: fam = dim + 6.0; break;
    case MC_FAMILY_ABS_LINEAR: fam = dim + 2.0; break;
    case MC_FAMILY_GAUSSIAN: fam = 3.0 * dim + 5.0; break;
    case MC_FAMILY_POLY_PRODUCT: fam = 8.0 * dim; break;
    default: fam = 40.0; break;  // run-time family: unknown, priced as a few transcendentals
    }
    double c = philox + dim + fam + 4.0;
    if (precision == MC_PREC_FP64) c *= 3.0;
    return c;
}

// ---------------------------------------------------------------- context state

struct Request;

struct FnState {
    uint32_t slot;        // device function slot
    uint32_t seg_log2;
    uint32_t n_tiles;
    uint32_t next_tile;   // next tile to put into a launch
    uint64_t part0;       // first partial slot
    double tile_cost;
    bool f64;             // evaluated by the FP64 kernel (requested, or promoted from FP32)
    bool needs_upload;    // record packed into the host mirror, not yet on the device
    uint32_t token;       // resident engine: the current run's token and record arena position
    uint32_t rec;
    bool done;            // its final result is in
};

struct Request {
    uint64_t id;
    int32_t precision;
    std::vector<mc_function> fns;     // caller's table (copied at submit); empty for a grid
    bool grid = false;                // records are built on the device from `spec`
    GridSpec spec{};
    uint64_t n = 0;                   // functions in the request
    size_t count() const { return (size_t)n; }
    mc_function at(size_t i) const
    {
        if (!grid) return fns[i];
        mc_function f;
        grid_function(spec.base, spec.axes, spec.n_axes, i, &f);
        return f;
    }
    std::vector<FnState> st;
    std::vector<mc_result> results;
    std::vector<uint32_t> order;      // functions by descending per-tile cost
    uint32_t order_pos = 0;           // next function in `order` with tiles left
    std::vector<uint32_t> redo;       // functions promoted from FP32 to FP64, to run again
    uint32_t redo_pos = 0;
    uint64_t part_base = 0, part_count = 0;
    uint32_t slot_base = 0;
    bool admitted = false;
    bool grid_packed = false;         // a grid's records have been built on the device
    hipEvent_t uploaded = nullptr;    // upload of the packed records (library upload stream)
    uint32_t fns_done = 0;
    uint64_t tiles_total = 0, tiles_launched = 0;
    double work_left = 0.0;           // estimated cost of the tiles not yet launched
    bool aborted = false;
    bool lost = false;                // part of its work went to a launch that failed after handing
                                      // finalize records to kernels: it completes with MC_ERR_HIP
    uint32_t n_promoted = 0;
    bool restored = false;            // built by mc_restore from a snapshot
    uint32_t fair_credit = 0;         // resident FAIR: tiles the request may still push this pass
    std::vector<Partial> staged;      // restored: its whole partial range, saved tiles filled in (uploaded at admission)
    std::vector<uint32_t> staged_counts;  // restored into a resident context: each function's tiles already run
    bool partials_pending = false;    // resident: admitted, saved partials not yet on the device
    bool cancelled = false;           // mc_cancel: no more of its work runs; it completes (MC_ERR_ABORTED)
                                      // once no kernel refers to its slots any more
};

// A function's consecutive tiles in one launch and the cost of one of them.
struct HostRun {
    double cost;
    TileRun run;
};

struct FinRef {
    Request* req;
    uint32_t index;
};

// What building a launch changes, kept so that a launch that fails before its
// finalize kernel is enqueued can be taken back.
struct TakeUndo {
    Request* req;
    uint32_t index;
    uint32_t next_tile;
    bool needs_upload;
};
struct RequestUndo {
    Request* req;
    uint32_t order_pos, redo_pos;
    uint64_t tiles_launched;
    double work_left;
};

// Timing events of one launch.  They are read once the runtime reports them
// complete, which can be well after the launch has published its results, so
// they come from a pool of their own rather than from the launch slot.
struct EvSet {
    hipEvent_t start = nullptr, mid = nullptr, main = nullptr, done = nullptr;
    bool main_is_mid = false;  // no FP64 or run-time family kernel ran: `mid` ends the main kernels
    bool pending = false;   // recorded, not yet read into the statistics
    bool graphed = false;
    bool released = false;  // the launch that recorded it has been reaped
};
constexpr size_t kEvPoolMax = 256;

// Staging of one launch: a device block and a pinned (fine-grained) host block:
//   device [results area | LaunchDesc + counters (kDescBytes) | finalize records | tile list]
//   host   [results area | LaunchDesc + counters (kDescBytes) | finalize records | tile runs]
// The host writes the descriptor (counters zeroed), the finalize records and
// one run per function with tiles in the launch (16 + 32 bytes per function,
// not 16 per tile); the stage kernel copies descriptor and records to the
// device block and expands the runs into the tile list, one contiguous part
// per kernel.  The publish kernel writes the launch's n_fins results into the
// end of the host block's results area (right before the descriptor) and the
// counters after the host copy of the descriptor, then the launch's sequence
// number into the slot's done word.
struct LaunchSlot {
    uint8_t* d_block = nullptr;     // device
    uint8_t* h_block = nullptr;     // pinned host
    uint8_t* h_block_dev = nullptr; // device address of h_block
    LaunchDesc* d_desc = nullptr;   // d_block + results area (fixed: captured graphs use it)
    hipStream_t stream = nullptr;   // stream of the slot's last launch
    EvSet* ev = nullptr;            // events of the slot's last launch
    hipGraphExec_t graph = nullptr;
    bool in_flight = false;
    bool graphed = false;             // this launch replayed the slot's graph
    uint64_t seq = 0;
    uint32_t n_tiles = 0, n_fins = 0;
    std::vector<Fin> fv;                // finalize records while the launch is built
    std::vector<HostRun> runs[kMaxKernels];  // each kernel's tile runs while the launch is built
    uint32_t n_runs = 0;
    uint32_t tile_begin[kMaxKernels] = {}, tile_count[kMaxKernels] = {};
    uint64_t n_samples = 0;             // integrand evaluations in this launch's tiles
    std::vector<FinRef> fin_refs;
    std::vector<Request*> touched;  // requests with tiles in this launch
    std::vector<TakeUndo> undo;     // function states before this launch took their tiles
};

// Resident engine (MC_RESIDENT).  Host side of the ring, the record arena and
// the runs whose chunks have been pushed.
constexpr uint32_t kRingEntries = 1u << 16;   // ring entries (power of two)
constexpr uint32_t kIdlePolls = 30000;        // a workgroup's polls for its entry (~0.1 s) before the launch stops
constexpr uint32_t kReadyPolls = 400000;      // polls of a record's ready word (~0.1 s) before a chunk is given up
constexpr uint32_t kLeaderEvery = 8;          // one workgroup in 8 reads the host's control word
constexpr uint32_t kArenaScan = 64;           // arena positions tried per new run while a launch runs

struct ResRun {
    Request* req;
    uint32_t index;  // function of the request
    uint32_t slot;
    uint32_t token;
    uint32_t rec;
};

struct ResidentState {
    bool on = false;
    hipStream_t stream = nullptr;
    uint32_t grid = 0;             // workgroups per launch
    uint64_t backlog = 0;          // tiles the ring may hold that no workgroup has read yet
    uint64_t unread_tiles = 0;     // tiles of the entries [acked, pushed)
    uint64_t tiles_waiting = 0;    // tiles of admitted requests not yet pushed
    bool active_dirty = false;     // the active list may be out of SRPT order
    size_t fair_pos = 0;           // FAIR: where the next pass over the active list starts
    // pinned, fine-grained host block
    uint8_t* h_block = nullptr;
    uint8_t* h_block_dev = nullptr;
    Chunk* ring = nullptr;
    uint64_t* ack = nullptr;
    uint64_t* ctl = nullptr;
    uint32_t* exit_word = nullptr;
    uint64_t* stage = nullptr;     // start values of a launch: tickets, control word, workgroups
    DevResult* results = nullptr;  // per function slot
    uint32_t* done = nullptr;      // per function slot
    // device
    ResidentDesc* d_desc = nullptr;
    uint64_t* d_pos = nullptr;
    uint32_t* d_running = nullptr;
    uint32_t* d_bad = nullptr;
    uint32_t* d_tiles_done = nullptr;
    uint32_t n_arena = 0;
    // ring positions: [0, acked) read by workgroups (or dropped by an abort), [acked, pushed) waiting
    uint64_t pushed = 0, acked = 0;
    uint32_t epoch = 0;            // of the last launch (the first is 1)
    bool live = false;             // the last launch has not stored its exit word yet
    bool stopping = false;         // the host asked it to stop
    bool flush = false;            // no arena position free until the running launch ends
    uint32_t next_token = 0;
    uint32_t cursor = 0;           // next arena position to try
    std::vector<uint32_t> arena_epoch;  // per position: the last launch that may have read it
    std::vector<uint8_t> arena_busy;    // per position: used by a run whose result is not in
    std::vector<ResRun> runs;           // runs with chunks pushed whose result is not in
    // with run-time families registered: the resident kernel compiled with them
    hipModule_t user_module = nullptr;
    hipFunction_t user_kernel = nullptr;
};

constexpr size_t kDescBytes = 512;  // LaunchDesc followed by its counters (zero padded)
static_assert(kUserFamily0 == (uint32_t)MC_FAMILY_USER0 && kMaxUserFamilies == MC_MAX_USER_FAMILIES,
              "run-time family ids");
static_assert(sizeof(LaunchDesc) + kNumCounters * sizeof(uint32_t) <= kDescBytes, "launch descriptor size");

}  // namespace

struct mc_ctx {
    mc_config cfg{};
    bool validate_only = false;
    bool use_graph = true;
    int device = 0;
    int num_cus = 0;
    std::string device_name;  // gcnArchName (keys the tuning cache)
    std::string err;

    // capacities
    uint32_t max_functions = 0;
    uint64_t max_partials = 0;
    uint32_t tile_cap = 0;   // per launch per precision
    uint32_t fin_cap = 0;
    uint64_t slot_res_bytes = 0;  // results area of a launch slot's block (fin_cap results, 256-aligned)
    uint64_t slot_bytes = 0;      // whole block

    // device memory
    uint8_t* scratch = nullptr;   // device address of the static `scratch` array on this device
    bool owns_memory = true;
    void* mem_base = nullptr;
    uint64_t mem_bytes = 0;
    DevFn* d_fns = nullptr;
    Partial* d_partials = nullptr;
    LaunchSlot slots[kLaunchSlots];
    uint32_t* d_abort_word = nullptr;  // device word the persistent kernels poll
    uint32_t* h_words = nullptr;       // pinned {0, 1}: sources for setting / clearing it
    uint32_t* h_done = nullptr;        // pinned fine-grained: one done word per launch slot (16 words apart)
    uint32_t* h_done_dev = nullptr;    // its device address
    DevFn* h_fns = nullptr;            // pinned fine-grained host mirror of the function table (records
                                       // are packed here at admission and uploaded from here)
    DevFn* h_fns_dev = nullptr;        // its device address (read by the stage kernel)
    std::vector<std::unique_ptr<EvSet>> ev_pool;
    std::vector<EvSet*> ev_free;
    std::deque<EvSet*> ev_pending;     // recorded sets, oldest first
    bool abort_requested = false;
    uint64_t abort_below = 0;          // the abort covers the requests with smaller ids

    RangeAlloc fn_alloc, part_alloc;

    // tuning
    uint32_t blocks_per_cu32 = 4, blocks_per_cu64 = 2;
    uint8_t seg_log2[2][kNumFamilies][kMaxDim];

    // requests
    uint64_t next_id = 1;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> requests;
    std::deque<Request*> pending;     // submitted, not admitted (FIFO)
    std::deque<Request*> active;      // admitted with tiles not yet launched
    std::deque<uint64_t> completed;   // request ids finished since the last mc_poll
    hipStream_t upload_stream = nullptr;
    uint32_t policy = MC_SCHED_FAIR;
    bool promote = true;
    uint64_t launch_seq = 0;
    double last_main_ms = 0.0, last_fin_ms = 0.0;
    bool have_timing = false;
    mc_stats stats{};

    // run-time compiled families (hipRTC): module and FP32/FP64 kernels of each
    struct UserFamily {
        hipModule_t module = nullptr;
        hipFunction_t kernel[2] = {nullptr, nullptr};
        uint32_t blocks_per_cu[2] = {1, 1};
    };
    UserFamily user[kMaxUserFamilies];
    uint32_t n_user = 0;
    std::vector<std::string> user_src;  // their sources (a resident kernel is compiled with all of them)

    ResidentState res;
};

namespace {

mc_status fail(mc_ctx* ctx, mc_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    g_thread_error = buf;
    log_msg(1, "error %d: %s", (int)st, buf);
    return st;
}

// An allocation the runtime refuses is reported as such, whichever call made it.
mc_status fail_hip(mc_ctx* ctx, const HipError& e)
{
    const mc_status st = e.e == hipErrorOutOfMemory ? MC_ERR_OUT_OF_MEMORY : MC_ERR_HIP;
    return fail(ctx, st, "%s failed: %s", e.what, hipGetErrorString(e.e));
}

uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

struct Layout {
    uint64_t fns, partials, slots, slot_res_bytes, slot_bytes, abort_word, total;
    // resident contexts: descriptor and counters, per-slot words, ready words, record arena
    uint64_t res_desc, res_tiles_done, res_slot_err, res_ready, res_arena;
    uint32_t n_arena;
};

// Record arena of a resident context: eight positions per function slot, at
// least 8192 and at most 2^20 (1 GiB).  A run holds one position until its
// result is in, and a position read by the running launch waits for the next
// one, so every (arena size - function slots) new runs the kernel is stopped
// and started again, which stalls the runs in flight for up to a chunk; a
// large arena makes that rare (a serving mix of 4 x 10^5 functions runs
// through 2^20 positions without it).
uint32_t arena_positions(uint32_t max_functions)
{
    return (uint32_t)std::min<uint64_t>(std::max<uint64_t>(8ull * max_functions, 8192), 1u << 20);
}

Layout compute_layout(uint32_t max_functions, uint64_t max_partials, uint32_t tile_cap, uint32_t fin_cap,
                      bool resident)
{
    Layout L{};
    uint64_t off = 0;
    if (resident) {
        // no launch slots and no per-slot table: records live in the arena
        L.n_arena = arena_positions(max_functions);
        L.partials = off;
        off = align_up(off + max_partials * sizeof(Partial), 256);
        L.res_desc = off;
        off += 512;  // ResidentDesc, then tickets and control word, workgroups, bad-chunk count
        L.res_tiles_done = off;
        off = align_up(off + (uint64_t)max_functions * sizeof(uint32_t), 256);
        L.res_slot_err = off;
        off = align_up(off + (uint64_t)max_functions * sizeof(uint32_t), 256);
        L.res_ready = off;
        off = align_up(off + (uint64_t)L.n_arena * sizeof(uint32_t), 256);
        L.res_arena = off;
        off += (uint64_t)L.n_arena * sizeof(DevFn);
        L.abort_word = off;
        off = align_up(off + sizeof(uint32_t), 256);
        L.total = off;
        return L;
    }
    L.fns = off;
    off = align_up(off + (uint64_t)max_functions * sizeof(DevFn), 256);
    L.partials = off;
    off = align_up(off + max_partials * sizeof(Partial), 256);
    L.slots = off;
    L.slot_res_bytes = align_up((uint64_t)fin_cap * sizeof(DevResult), 256);
    // device: descriptor, finalize records, tile list; host: descriptor, finalize
    // records, tile runs (at most one per function slot)
    L.slot_bytes = align_up(L.slot_res_bytes + kDescBytes + (uint64_t)fin_cap * sizeof(Fin) +
                                std::max<uint64_t>((uint64_t)tile_cap * sizeof(Tile), (uint64_t)fin_cap * sizeof(TileRun)),
                            256);
    off += kLaunchSlots * L.slot_bytes;
    L.abort_word = off;
    off = align_up(off + sizeof(uint32_t), 256);
    L.total = off;
    return L;
}

void resolve_capacities(const mc_config& cfg, uint32_t* max_functions, uint64_t* max_partials, uint32_t* tile_cap,
                        uint32_t* fin_cap)
{
    *max_functions = cfg.max_functions ? cfg.max_functions : (1u << 16);
    *tile_cap = cfg.max_tiles_per_run ? cfg.max_tiles_per_run : (1u << 20);
    *fin_cap = *max_functions;
    if (cfg.max_partials) {
        *max_partials = cfg.max_partials;
    } else {
        *max_partials = 1ull << 22;
        if (cfg.mem_budget_bytes) {
            Layout fixed = compute_layout(*max_functions, 0, *tile_cap, *fin_cap, (cfg.flags & MC_RESIDENT) != 0);
            if (cfg.mem_budget_bytes > fixed.total + 4096)
                *max_partials = std::min<uint64_t>(*max_partials, (cfg.mem_budget_bytes - fixed.total - 4096) / sizeof(Partial));
            else
                *max_partials = 1;
        }
    }
}

// Tiles of one function for a given seg_log2.
uint32_t tiles_for(uint32_t n_segments, uint32_t seg_log2)
{
    const uint32_t per_tile = (uint32_t)kBlockWaves << seg_log2;
    return (n_segments + per_tile - 1) / per_tile;
}

// Give an admitted request's function slots and partial range back.
void release_slots(mc_ctx* ctx, Request* r)
{
    if (!r->admitted) return;
    ctx->fn_alloc.release(r->slot_base, r->count());
    ctx->part_alloc.release(r->part_base, r->part_count);
    r->admitted = false;
}

// Everything a finished request holds: its pending upload, a restored
// request's saved partials and counts, its slots.
void free_request_resources(mc_ctx* ctx, Request* r)
{
    if (r->uploaded) {
        // an upload into its slots still on the upload stream (a request aborted
        // or cancelled before a launch waited for it) lands before the slots
        // are handed to another request; otherwise it is long complete
        quiet(hipEventSynchronize(r->uploaded));
        quiet(hipEventDestroy(r->uploaded));
        r->uploaded = nullptr;
    }
    std::vector<Partial>().swap(r->staged);
    std::vector<uint32_t>().swap(r->staged_counts);
    release_slots(ctx, r);
}

bool has_work(const Request* r)
{
    return r->order_pos < r->order.size() || r->redo_pos < r->redo.size();
}

// No more of request r's work is handed to the GPU.
void drop_work(Request* r)
{
    r->order_pos = (uint32_t)r->order.size();
    r->redo_pos = (uint32_t)r->redo.size();
    r->tiles_launched = r->tiles_total;
    r->work_left = 0.0;
}

// Complete request r as aborted (mc_abort, mc_cancel): results already in
// stay, every other one carries MC_ERR_ABORTED, its slots are released and its
// id is reported complete.  Nothing on the GPU may refer to its slots any more.
void complete_aborted(mc_ctx* ctx, Request* r)
{
    for (uint32_t i = 0; i < r->count(); ++i) {
        if (r->st[i].done) continue;
        mc_result& out = r->results[i];
        std::memset(&out, 0, sizeof out);
        out.n = r->grid ? r->spec.base.n_samples : r->fns[i].n_samples;
        out.status = MC_ERR_ABORTED;
        out.precision = (uint32_t)r->precision;
    }
    r->aborted = true;
    r->fns_done = (uint32_t)r->count();
    drop_work(r);
    free_request_resources(ctx, r);
    ctx->completed.push_back(r->id);
}

// Whether an FP32-evaluated result must be computed again in FP64.  `scale`
// is the factor the FP32 path takes out of every sample (f = scale * g, the
// sums scaled in FP64), so only g passes through FP32 arithmetic.
// * Range: every g and g^2 is an FP32 value, summed in FP32 over 64 samples
//   per lane before the FP64 reduction.  |g| beyond about 2^60 overflows those
//   sums (non-finite S1 or S2); below about 2^-60 the squares underflow (mean
//   of g^2 under 2^-120, or zero -- also when g itself rounds to 0 in FP32, so
//   an integrand that is zero in FP32 everywhere with a nonzero scale is
//   checked in FP64 too).  A zero scale means f == 0 exactly.
// * Accuracy: FP32 evaluation rounds each sample to about 2^-24 of its size;
//   a bias of a few such units of the RMS value must stay below 0.01 of the
//   standard error, i.e. sigma / rms must exceed 100 * 4 * 2^-24 * sqrt(N).
//   Below that (nearly constant integrands) the FP32 result cannot be
//   trusted to that accuracy.
bool fp32_unresolved(const mc_result& r, double scale)
{
    const double n = (double)r.n;
    if (!(n >= 2.0)) return false;
    if (!std::isfinite(r.sum_f) || !std::isfinite(r.sum_f2)) return true;
    if (scale == 0.0) return false;
    const double rms2 = r.sum_f2 / n;
    if (!(rms2 / (scale * scale) >= 0x1p-120)) return true;
    const double var = (r.sum_f2 - r.sum_f * r.sum_f / n) / (n - 1.0);
    const double ratio = var > 0.0 ? std::sqrt(var / rms2) : 0.0;
    return ratio < 400.0 * std::ldexp(1.0, -24) * std::sqrt(n);
}

void promote_to_fp64(mc_ctx* ctx, Request* r, uint32_t fi)
{
    FnState& fs = r->st[fi];
    fs.f64 = true;
    fs.next_tile = 0;
    r->tiles_total += fs.n_tiles;
    const mc_function f = r->at(fi);
    fs.tile_cost = sample_cost(f.family, f.dim, MC_PREC_FP64) *
                   (double)std::min<uint64_t>(f.n_samples, (uint64_t)kSegSamples * ((uint64_t)kBlockWaves << fs.seg_log2));
    r->work_left += fs.tile_cost * fs.n_tiles;
    // the slot's previous upload has completed (its FP32 result came back); the
    // FP64 record goes up with the first launch of its tiles
    pack_function(f, MC_PREC_FP64, &ctx->h_fns[fs.slot]);
    fs.needs_upload = true;
    const bool was_active = has_work(r);
    r->redo.push_back(fi);
    r->n_promoted++;
    ctx->stats.promoted++;
    log_msg(2, "request %llu function %u: FP32 result cannot be trusted, running it in FP64",
            (unsigned long long)r->id, fi);
    if (!was_active) ctx->active.push_back(r);
    if (ctx->res.on) {
        ctx->res.tiles_waiting += fs.n_tiles;
        ctx->res.active_dirty = true;
    }
}

// Read a launch's timing events into the statistics.  block = false: only if
// the runtime already reports them complete.
void collect_timing(mc_ctx* ctx, EvSet& e, bool block)
{
    if (!e.pending) return;
    const hipError_t q = block ? hipEventSynchronize(e.done) : hipEventQuery(e.done);
    quiet(q);
    if (q == hipErrorNotReady) return;
    e.pending = false;
    if (q != hipSuccess) return;  // timing lost; results are unaffected
    float a = 0.f, a32 = 0.f, b = 0.f, g = 0.f;
    if (e.graphed) {
        const hipError_t e1 = hipEventElapsedTime(&g, e.start, e.done);
        quiet(e1);
        if (e1 == hipSuccess) ctx->stats.graph_ms += g;
        return;
    }
    const hipEvent_t main = e.main_is_mid ? e.mid : e.main;
    const hipError_t e1 = hipEventElapsedTime(&a, e.start, main);
    const hipError_t e2 = hipEventElapsedTime(&a32, e.start, e.mid);
    const hipError_t e3 = hipEventElapsedTime(&b, main, e.done);
    quiet(e1);
    quiet(e2);
    quiet(e3);
    if (e1 == hipSuccess && e2 == hipSuccess && e3 == hipSuccess) {
        ctx->last_main_ms = a;
        ctx->last_fin_ms = b;
        ctx->have_timing = true;
        ctx->stats.fp32_ms += a32;
        ctx->stats.fp64_ms += a - a32;
        ctx->stats.finalize_ms += b;
    }
}

// Read the pending sets of reaped launches, oldest first; block = false stops at
// the first one the runtime has not released yet.  Read sets return to the pool.
void collect_pending(mc_ctx* ctx, bool block)
{
    while (!ctx->ev_pending.empty()) {
        EvSet* e = ctx->ev_pending.front();
        if (!e->released) return;
        collect_timing(ctx, *e, block);
        if (e->pending) return;
        ctx->ev_pending.pop_front();
        ctx->ev_free.push_back(e);
    }
}

// Every reaped launch's timing (waits for the events).
void collect_all_timing(mc_ctx* ctx) { collect_pending(ctx, true); }

// A free event set for a new launch: reuses read sets, creates new ones up to
// kEvPoolMax, and only then waits for the oldest pending one.
EvSet* acquire_evset(mc_ctx* ctx)
{
    collect_pending(ctx, false);
    if (ctx->ev_free.empty() && ctx->ev_pool.size() >= kEvPoolMax) collect_pending(ctx, true);
    if (ctx->ev_free.empty()) {
        std::unique_ptr<EvSet> e(new EvSet());
        try {
            HIP_TRY(hipEventCreate(&e->start));
            HIP_TRY(hipEventCreate(&e->mid));
            HIP_TRY(hipEventCreate(&e->main));
            HIP_TRY(hipEventCreate(&e->done));
        } catch (const HipError&) {
            for (hipEvent_t x : {e->start, e->mid, e->main, e->done})
                if (x) quiet(hipEventDestroy(x));
            throw;
        }
        ctx->ev_free.push_back(e.get());
        ctx->ev_pool.push_back(std::move(e));
    }
    EvSet* e = ctx->ev_free.back();
    ctx->ev_free.pop_back();
    e->pending = false;
    e->released = false;
    return e;
}

bool any_in_flight(const mc_ctx* ctx)
{
    for (const auto& s : ctx->slots)
        if (s.in_flight) return true;
    return false;
}

// Whether a launch in flight still refers to request r (tiles or finalize records).
bool in_flight_refers(const mc_ctx* ctx, const Request* r)
{
    for (const auto& s : ctx->slots) {
        if (!s.in_flight) continue;
        for (const Request* t : s.touched)
            if (t == r) return true;
        for (const FinRef& f : s.fin_refs)
            if (f.req == r) return true;
    }
    return false;
}

uint32_t load_done(const mc_ctx* ctx, const LaunchSlot& s)
{
    const uint32_t* w = ctx->h_done + 16 * (&s - ctx->slots);
    return __atomic_load_n(w, __ATOMIC_ACQUIRE);
}

// Wait until the launch in `s` has published its results.  Spins, then yields,
// then sleeps in short steps; if the runtime reports the launch's last event
// complete while the done word still lags, that is an error (not a hang).
void wait_done(mc_ctx* ctx, LaunchSlot& s)
{
    const uint32_t want = (uint32_t)s.seq;
    for (uint64_t i = 0;; ++i) {
        if (load_done(ctx, s) == want) return;
        if (i < 4096) continue;
        if (i < 65536) {
            sched_yield();
            continue;
        }
        if ((i & 255) == 0) {
            const hipError_t q = hipEventQuery(s.ev->done);
            quiet(q);
            if (q != hipErrorNotReady) {
                if (load_done(ctx, s) == want) return;
                if (q != hipSuccess) throw HipError{q, "hipEventQuery(launch)"};
                throw HipError{hipErrorUnknown, "launch finished without publishing its results"};
            }
        }
        struct timespec ts{0, 20000};
        nanosleep(&ts, nullptr);
    }
}

// A function's result is in: store it, send an FP32 result that cannot be
// trusted to FP64, and complete the request with its last function.
void complete_function(mc_ctx* ctx, Request* req, uint32_t index, const DevResult& res, bool bad)
{
    if (req->cancelled) return;  // (it completes as aborted once nothing refers to it)
    mc_result& out = req->results[index];
    std::memcpy(&out, &res, sizeof(mc_result));
    if (bad) out.status = MC_ERR_HIP;
    // the host's own record of the precision decides (a result can be promoted
    // once); a device record that disagrees is an error
    const bool host_f64 = req->st[index].f64;
    if (out.status == MC_OK && out.precision != (host_f64 ? (uint32_t)MC_PREC_FP64 : (uint32_t)MC_PREC_FP32_EVAL)) {
        out.status = MC_ERR_HIP;
        ctx->err = "a result came back in another precision than its function was scheduled in";
    }
    if (out.status == MC_OK && !host_f64 && ctx->promote && !req->lost &&
        fp32_unresolved(out, req->grid ? fp32_scale(req->at(index)) : fp32_scale(req->fns[index]))) {
        promote_to_fp64(ctx, req, index);
        return;
    }
    if (out.status != MC_OK) req->aborted = true;
    req->st[index].done = true;
    req->fns_done++;
    if (req->fns_done == req->count()) {
        free_request_resources(ctx, req);
        ctx->completed.push_back(req->id);
    }
}

// Collect finished launches (oldest first): scatter their results into the
// requests.  wait = 0: only what has completed; 1: wait for the oldest launch
// in flight first; 2: wait for every launch in flight.
void reap(mc_ctx* ctx, int wait)
{
    bool waited = false;
    for (;;) {
        LaunchSlot* oldest = nullptr;
        for (auto& s : ctx->slots)
            if (s.in_flight && (!oldest || s.seq < oldest->seq)) oldest = &s;
        if (!oldest) return;
        const bool block = wait == 2 || (wait == 1 && !waited);
        waited = true;
        if (load_done(ctx, *oldest) != (uint32_t)oldest->seq) {
            if (!block) return;
            wait_done(ctx, *oldest);
        }
        LaunchSlot& s = *oldest;
        const uint8_t* hdesc = s.h_block + ctx->slot_res_bytes;
        const uint32_t* cnt = (const uint32_t*)(hdesc + sizeof(LaunchDesc));
        const DevResult* hres = (const DevResult*)hdesc - s.n_fins;
        const uint32_t bad = cnt[kCounterBadRecords];
        if (bad != 0) {
            char buf[160];
            snprintf(buf, sizeof buf, "launch %llu: %u tile/finalize records failed the kernels' bounds checks",
                     (unsigned long long)s.seq, bad);
            ctx->err = buf;
        }
        for (uint32_t i = 0; i < s.n_fins; ++i) {
            const FinRef& fr = s.fin_refs[i];
            complete_function(ctx, fr.req, fr.index, hres[i], bad != 0);
        }
        {
            s.ev->released = true;
            ctx->stats.launches++;
            for (int k = 0; k < kMaxKernels; ++k) {
                if (k % 2 == 0) ctx->stats.tiles32 += s.tile_count[k];
                else ctx->stats.tiles64 += s.tile_count[k];
            }
            ctx->stats.functions += s.n_fins;
            ctx->stats.samples += s.n_samples;
            ctx->stats.bad_records += bad;
        }
        s.in_flight = false;
        // cancelled requests this launch referred to complete once no other launch does
        std::vector<Request*> refs(s.touched.begin(), s.touched.end());
        for (const FinRef& fr : s.fin_refs) refs.push_back(fr.req);
        s.fin_refs.clear();
        s.touched.clear();
        for (Request* r : refs)
            if (r->cancelled && r->fns_done < r->count() && !in_flight_refers(ctx, r)) complete_aborted(ctx, r);
    }
}

// Move pending requests into device slots while they fit (FIFO).  With no
// launch in flight the records go up at once on the library's upload stream
// (launches that use the request wait for its upload event); otherwise a copy
// or kernel on another stream would wait for the running persistent kernels
// to free their compute units, so each record goes up with the stage kernel
// of the first launch that runs its tiles, and a grid's records are built in
// the launch stream right before it.  A resident context packs every record
// into the mirror (grids too, on the host): the first chunk of each run copies
// it to the device, so admission enqueues nothing.
void admit(mc_ctx* ctx)
{
    bool idle = true;
    for (const auto& sl : ctx->slots)
        if (sl.in_flight) idle = false;
    while (!ctx->pending.empty()) {
        if (ctx->res.on) {
            Request* r = ctx->pending.front();
            const uint64_t nf = r->count();
            uint64_t parts = 0;
            for (auto& st : r->st) parts += st.n_tiles;
            uint64_t slot_off = 0, part_off = 0;
            if (!ctx->fn_alloc.alloc(nf, &slot_off)) return;
            if (!ctx->part_alloc.alloc(parts, &part_off)) {
                ctx->fn_alloc.release(slot_off, nf);
                return;
            }
            r->slot_base = (uint32_t)slot_off;
            r->part_base = part_off;
            r->part_count = parts;
            uint64_t p = part_off;
            for (uint32_t i = 0; i < nf; ++i) {
                FnState& fs = r->st[i];
                fs.slot = (uint32_t)slot_off + i;
                fs.part0 = p;
                p += fs.n_tiles;
                pack_function(r->at(i), fs.f64 ? MC_PREC_FP64 : MC_PREC_FP32_EVAL, &ctx->h_fns[fs.slot]);
            }
            r->admitted = true;
            r->grid_packed = true;
            r->partials_pending = !r->staged.empty();  // (copied by res_upload_restored)
            ctx->pending.pop_front();
            ctx->active.push_back(r);
            log_msg(3, "request %llu admitted: %llu functions, %llu tiles", (unsigned long long)r->id,
                    (unsigned long long)nf, (unsigned long long)r->tiles_total);
            ctx->res.tiles_waiting += r->tiles_total - r->tiles_launched;
            ctx->res.active_dirty = true;
            continue;
        }
        Request* r = ctx->pending.front();
        const uint64_t nf = r->count();
        uint64_t parts = 0;
        for (auto& s : r->st) parts += s.n_tiles;
        uint64_t slot_off = 0, part_off = 0;
        if (!ctx->fn_alloc.alloc(nf, &slot_off)) return;
        if (!ctx->part_alloc.alloc(parts, &part_off)) {
            ctx->fn_alloc.release(slot_off, nf);
            return;
        }
        r->slot_base = (uint32_t)slot_off;
        r->part_base = part_off;
        r->part_count = parts;
        uint64_t p = part_off;
        for (uint32_t i = 0; i < nf; ++i) {
            r->st[i].slot = (uint32_t)slot_off + i;
            r->st[i].part0 = p;
            p += r->st[i].n_tiles;
        }
        r->admitted = true;  // from here on the slots are released with the request
        bool enqueued = false;
        try {
            if (r->grid) {
                // a restored grid's rows already promoted to FP64 take host-packed
                // FP64 records, copied by their first launch after the grid's
                // device-packed ones, as when they were promoted
                if (r->restored && r->spec.precision != MC_PREC_FP64)
                    for (uint64_t i = 0; i < nf; ++i)
                        if (r->st[i].f64 && r->st[i].next_tile < r->st[i].n_tiles) {
                            pack_function(r->at(i), MC_PREC_FP64, &ctx->h_fns[slot_off + i]);
                            r->st[i].needs_upload = true;
                        }
                // records built on the device from the grid spec: no table crosses PCIe
                if (idle) {
                    DevFn* out = ctx->d_fns + slot_off;
                    void* args[] = {&r->spec, &out};
                    enqueued = true;
                    HIP_TRY(hipLaunchKernel(pack_grid_kernel_ptr(), dim3((unsigned)((nf + 255) / 256)), dim3(256),
                                            args, 0, ctx->upload_stream));
                    r->grid_packed = true;
                }
            } else {
                // records packed into the slots' part of the pinned mirror (whose
                // previous uploads completed before those slots were released)
                for (uint64_t i = 0; i < nf; ++i)
                    pack_function(r->fns[i], r->st[i].f64 ? MC_PREC_FP64 : MC_PREC_FP32_EVAL,
                                  &ctx->h_fns[slot_off + i]);
                if (idle) {
                    enqueued = true;
                    HIP_TRY(hipMemcpyAsync(ctx->d_fns + slot_off, ctx->h_fns + slot_off, nf * sizeof(DevFn),
                                           hipMemcpyHostToDevice, ctx->upload_stream));
                } else {
                    for (uint64_t i = 0; i < nf; ++i) r->st[i].needs_upload = true;
                }
            }
            // a restored request's saved partials go up on the upload stream;
            // launches with its tiles wait for the upload event
            if (!r->staged.empty()) {
                enqueued = true;
                HIP_TRY(hipMemcpyAsync(ctx->d_partials + part_off, r->staged.data(), parts * sizeof(Partial),
                                       hipMemcpyHostToDevice, ctx->upload_stream));
            }
            if (idle || !r->staged.empty()) {
                HIP_TRY(hipEventCreateWithFlags(&r->uploaded, hipEventDisableTiming));
                HIP_TRY(hipEventRecord(r->uploaded, ctx->upload_stream));
            }
        } catch (const HipError&) {
            // the request stays first in the queue, unadmitted, and is admitted
            // again later (a restored one keeps its saved partials for that);
            // an upload already handed to the stream finishes before its slots
            // can be handed to anyone else
            if (enqueued) quiet(hipStreamSynchronize(ctx->upload_stream));
            if (r->uploaded) {
                quiet(hipEventDestroy(r->uploaded));
                r->uploaded = nullptr;
            }
            for (uint64_t i = 0; i < nf; ++i) r->st[i].needs_upload = false;
            r->grid_packed = false;
            release_slots(ctx, r);
            throw;
        }
        ctx->pending.pop_front();
        ctx->active.push_back(r);
        log_msg(3, "request %llu admitted: %llu functions, %llu tiles", (unsigned long long)r->id,
                (unsigned long long)nf, (unsigned long long)r->tiles_total);
    }
}

void capture_graph(mc_ctx* ctx, LaunchSlot& s);

// The kernels of a launch: stage, the batched kernels (built-in FP32 and FP64,
// then those of run-time families with tiles), finalize, publish.  Direct
// launches bracket the batched kernels and the finalize with timing events; a
// captured graph holds the kernels only and is timed as a whole from outside
// (events recorded inside captured graphs are not reliable timing sources).
// *progress: 1 once the stage kernel is handed to the stream, 2 once the
// finalize kernel is (from then on the launch's finalize records are in use).
void enqueue_kernels(mc_ctx* ctx, LaunchSlot& s, hipStream_t stream, bool events, int* progress)
{
    LaunchDesc* dd = s.d_desc;
    void* args[] = {&dd};
    {
        // staging: descriptor, counters, tiles and finalize records, host -> device
        const uint8_t* src = s.h_block_dev + ctx->slot_res_bytes;
        uint8_t* dst = s.d_block + ctx->slot_res_bytes;
        uint64_t cap = kDescBytes + (uint64_t)ctx->fin_cap * sizeof(Fin);
        uint32_t tile_cap = ctx->tile_cap;
        const DevFn* mirror = ctx->h_fns_dev;
        DevFn* fns = ctx->d_fns;
        uint32_t n_fns = ctx->max_functions;
        void* sargs[] = {&src, &dst, &cap, &tile_cap, &mirror, &fns, &n_fns};
        *progress = std::max(*progress, 1);
        HIP_TRY(hipLaunchKernel(stage_kernel_ptr(), dim3(ctx->num_cus * 2), dim3(256), sargs, 0, stream));
    }
    EvSet* e = s.ev;
    // a graph holds every built-in kernel (an empty one exits at once);
    // direct launches skip kernels without tiles
    if (events) HIP_TRY(hipEventRecord(e->start, stream));
    if (!events || s.tile_count[kKernelBuiltin32] != 0)
        HIP_TRY(hipLaunchKernel(batched_kernel_ptr(false), dim3(ctx->num_cus * ctx->blocks_per_cu32),
                                dim3(kBlockThreads), args, 0, stream));
    if (events) HIP_TRY(hipEventRecord(e->mid, stream));
    if (!events || s.tile_count[kKernelBuiltin64] != 0)
        HIP_TRY(hipLaunchKernel(batched_kernel_ptr(true), dim3(ctx->num_cus * ctx->blocks_per_cu64),
                                dim3(kBlockThreads), args, 0, stream));
    // run-time families: kernels with no tiles in this launch are skipped
    bool more = events && s.tile_count[kKernelBuiltin64] != 0;
    for (uint32_t u = 0; u < ctx->n_user; ++u)
        for (int p = 0; p < 2; ++p) {
            if (s.tile_count[2 + 2 * u + p] == 0) continue;
            const mc_ctx::UserFamily& uf = ctx->user[u];
            more = more || events;
            HIP_TRY(hipModuleLaunchKernel(uf.kernel[p], ctx->num_cus * uf.blocks_per_cu[p], 1, 1, kBlockThreads, 1, 1,
                                          0, stream, args, nullptr));
        }
    // (each event between kernels widens the gap between them by a few
    // microseconds: one is recorded only where a kernel ran after `mid`, and
    // the launch's `done` event, recorded after the publish kernel, ends the
    // finalize-and-publish interval)
    if (more) HIP_TRY(hipEventRecord(e->main, stream));
    if (events) e->main_is_mid = !more;
    *progress = 2;
    HIP_TRY(hipLaunchKernel(finalize_kernel_ptr(), dim3(ctx->num_cus * 2), dim3(kBlockThreads), args, 0, stream));
    HIP_TRY(hipLaunchKernel(publish_kernel_ptr(), dim3(1), dim3(1024), args, 0, stream));
}

void capture_graph(mc_ctx* ctx, LaunchSlot& s)
{
    if (s.graph) {
        quiet(hipGraphExecDestroy(s.graph));
        s.graph = nullptr;
    }
    hipStream_t cs;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    bool capturing = false;
    try {
        HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        capturing = true;
        int progress = 0;  // (nothing runs while capturing)
        enqueue_kernels(ctx, s, cs, false, &progress);
        capturing = false;
        HIP_TRY(hipStreamEndCapture(cs, &g));
        HIP_TRY(hipGraphInstantiate(&s.graph, g, nullptr, nullptr, 0));
    } catch (...) {
        if (capturing) quiet(hipStreamEndCapture(cs, &g));  // leave capture mode before the stream goes
        if (g) quiet(hipGraphDestroy(g));
        quiet(hipStreamDestroy(cs));
        throw;
    }
    quiet(hipGraphDestroy(g));
    quiet(hipStreamDestroy(cs));
}

// Put up to `budget` tiles of request r into launch slot s (functions in
// descending per-tile cost), with a finalize record for every function whose
// last tile goes in.  Returns false when a capacity of the slot is exhausted.
bool take_tiles(mc_ctx* ctx, LaunchSlot& s, Request* r, uint64_t budget)
{
    uint64_t taken = 0;
    bool room = true;
    while (has_work(r)) {
        const bool in_order = r->order_pos < r->order.size();
        const uint32_t fi = in_order ? r->order[r->order_pos] : r->redo[r->redo_pos];
        FnState& fs = r->st[fi];
        const int kidx = kernel_index(r->grid ? r->spec.base.family : r->fns[fi].family, fs.f64);
        const uint64_t tile_samples = ((uint64_t)kBlockWaves << fs.seg_log2) * kSegSamples;
        const uint64_t fn_samples = r->grid ? r->spec.base.n_samples : r->fns[fi].n_samples;
        // the function's next tiles, as many as the launch and the share allow, in one run
        uint64_t take = fs.n_tiles - fs.next_tile;
        take = std::min<uint64_t>(take, ctx->tile_cap - s.n_tiles);
        take = std::min<uint64_t>(take, budget - std::min(budget, taken));
        if (take > 0 && s.n_runs >= ctx->fin_cap) take = 0;  // run records are full
        if (take > 0) {
            s.undo.push_back(TakeUndo{r, fi, fs.next_tile, fs.needs_upload});
            const uint64_t a = fs.next_tile, b = a + take;
            s.n_samples += std::min<uint64_t>(b * tile_samples, fn_samples) - a * tile_samples;
            HostRun hr;
            hr.cost = fs.tile_cost;
            hr.run = TileRun{fs.slot, (uint32_t)a, (uint32_t)take, fs.seg_log2, (uint32_t)fs.part0, 0u,
                             fs.needs_upload ? kRunUploadRecord : 0u, 0u};
            fs.needs_upload = false;
            s.runs[kidx].push_back(hr);
            s.n_runs++;
            s.n_tiles += (uint32_t)take;
            fs.next_tile = (uint32_t)b;
            r->tiles_launched += take;
            r->work_left = std::max(0.0, r->work_left - fs.tile_cost * (double)take);
            taken += take;
        }
        if (taken > 0 && (s.touched.empty() || s.touched.back() != r)) s.touched.push_back(r);
        if (fs.next_tile < fs.n_tiles) {
            room = s.n_tiles < ctx->tile_cap && s.n_runs < ctx->fin_cap;
            break;
        }
        if (s.n_fins >= ctx->fin_cap) {
            room = false;
            break;
        }
        s.fv.emplace_back();
        Fin& f = s.fv.back();
        f.fn = fs.slot;
        f.part0 = (uint32_t)fs.part0;
        f.n_tiles = fs.n_tiles;
        f.res = s.n_fins;
        s.fin_refs.push_back(FinRef{r, fi});
        s.n_fins++;
        if (in_order) r->order_pos++;
        else r->redo_pos++;
        if (has_work(r) && taken >= budget) break;
    }
    return room;
}

// A launch whose enqueueing failed after it took its tiles.  Kernels it did
// hand to the stream (progress > 0) are drained first, so that none of them
// still reads the slot's blocks or writes partials when they are used again,
// and the launch's sequence number, which its publish kernel may have stored
// in the slot's done word, is never reused.  Before its finalize kernel was
// enqueued (progress < 2) the take is undone: every request is as it was and
// the next launch takes the same tiles, whose partials it rewrites with the
// same values.  After that (finalize compacts partials in place), or if the
// stream cannot be drained, the work of every request in the launch is lost:
// those requests complete with MC_ERR_HIP and take no more launches.
void abandon_launch(mc_ctx* ctx, LaunchSlot& s, hipStream_t stream, int progress,
                    const std::vector<RequestUndo>& req_undo, const std::deque<Request*>& active_before)
{
    bool drained = true;
    if (progress > 0) {
        const hipError_t q = hipStreamSynchronize(stream);
        quiet(q);
        drained = q == hipSuccess;
        ctx->launch_seq++;
    }
    if (progress < 2 && drained) {
        for (auto it = s.undo.rbegin(); it != s.undo.rend(); ++it) {
            FnState& fs = it->req->st[it->index];
            fs.next_tile = it->next_tile;
            fs.needs_upload = it->needs_upload;
        }
        for (const RequestUndo& u : req_undo) {
            u.req->order_pos = u.order_pos;
            u.req->redo_pos = u.redo_pos;
            u.req->tiles_launched = u.tiles_launched;
            u.req->work_left = u.work_left;
        }
        ctx->active = active_before;
    } else {
        std::vector<Request*> lost(s.touched.begin(), s.touched.end());
        for (const FinRef& fr : s.fin_refs) lost.push_back(fr.req);
        for (Request* r : lost) {
            if (r->lost) continue;
            r->lost = true;
            r->order_pos = (uint32_t)r->order.size();
            r->redo_pos = (uint32_t)r->redo.size();
            r->tiles_launched = r->tiles_total;
            r->work_left = 0.0;
        }
        std::deque<Request*> keep;
        for (Request* r : ctx->active)
            if (!r->lost) keep.push_back(r);
        ctx->active.swap(keep);
    }
    s.n_tiles = s.n_fins = s.n_runs = 0;
    for (auto& v : s.runs) v.clear();
    s.fv.clear();
    s.fin_refs.clear();
    s.touched.clear();
    s.undo.clear();
}

// Build and enqueue one launch.  Returns false if nothing was launched (no
// admitted work, or no free launch slot).
bool launch(mc_ctx* ctx, hipStream_t stream, bool* no_slot)
{
    *no_slot = false;
    if (ctx->active.empty()) return false;
    LaunchSlot* slot = nullptr;
    for (auto& s : ctx->slots)
        if (!s.in_flight) {
            slot = &s;
            break;
        }
    if (!slot) {
        *no_slot = true;
        return false;
    }
    // what a launch may have to create (its event set, the slot's graph on
    // first use; neither depends on the launch's contents) is made before any
    // request's state changes, so that a failure leaves every request as it was
    EvSet* const evp = acquire_evset(ctx);
    LaunchSlot& s = *slot;
    if (ctx->use_graph && ctx->n_user == 0 && !s.graph) {
        try {
            capture_graph(ctx, s);
        } catch (const HipError&) {
            ctx->ev_free.push_back(evp);
            throw;
        }
    }
    s.n_tiles = s.n_fins = s.n_runs = 0;
    for (auto& v : s.runs) v.clear();
    s.fv.clear();
    s.n_samples = 0;
    s.fin_refs.clear();
    s.touched.clear();
    // FIFO fills the launch from the oldest request; FAIR gives every active
    // request an equal share first, so a small request never waits behind a
    // large one for more than one launch; SRPT fills it from the request with
    // the least work left (shortest remaining processing time first), which
    // under heavy-tailed request sizes shortens the wait of nearly every
    // request, the largest ones included, compared with equal sharing.
    const uint64_t n_active = ctx->active.size();
    const uint64_t share = ctx->policy == MC_SCHED_FAIR ? std::max<uint64_t>(ctx->tile_cap / n_active, 64)
                                                        : UINT64_MAX;
    if (ctx->policy == MC_SCHED_SRPT)
        std::stable_sort(ctx->active.begin(), ctx->active.end(),
                         [](const Request* a, const Request* b) { return a->work_left < b->work_left; });
    // what taking tiles changes, so that a launch that fails early can be taken back
    const std::deque<Request*> active_before = ctx->active;
    std::vector<RequestUndo> req_undo;
    req_undo.reserve(ctx->active.size());
    for (Request* r : ctx->active)
        req_undo.push_back(RequestUndo{r, r->order_pos, r->redo_pos, r->tiles_launched, r->work_left});
    s.undo.clear();
    std::deque<Request*> keep;
    for (Request* r : ctx->active) {
        if (has_work(r)) take_tiles(ctx, s, r, share);
        if (has_work(r)) keep.push_back(r);
    }
    ctx->active.swap(keep);
    if (s.n_tiles == 0 && s.n_fins == 0) {
        ctx->ev_free.push_back(evp);
        return false;
    }
    int progress = 0;  // 1: kernels of this launch are in the stream; 2: its finalize kernel is too
    try {
        // stage: finalize records after the descriptor, then the tile runs; the
        // stage kernel expands the runs into the device tile list, the kernels'
        // parts one after another
        uint8_t* const hdesc = s.h_block + ctx->slot_res_bytes;
        uint8_t* const ddesc = s.d_block + ctx->slot_res_bytes;
        Fin* const hfins = (Fin*)(hdesc + kDescBytes);
        TileRun* const hruns = (TileRun*)(hfins + s.n_fins);
        if (s.n_fins) std::memcpy(hfins, s.fv.data(), (size_t)s.n_fins * sizeof(Fin));
        {
            // Within a kernel's part, functions' runs go in descending tile cost, so
            // the last tiles each workgroup fetches are the cheapest (a short tail).
            // Results do not depend on the order.
            uint32_t off = 0, nr = 0;
            for (int k = 0; k < kMaxKernels; ++k) {
                s.tile_begin[k] = off;
                std::vector<HostRun>& rr = s.runs[k];
                std::stable_sort(rr.begin(), rr.end(), [](const HostRun& a, const HostRun& b) { return a.cost > b.cost; });
                for (HostRun& hr : rr) {
                    hr.run.dst = off;
                    hruns[nr++] = hr.run;
                    off += hr.run.count;
                }
                s.tile_count[k] = off - s.tile_begin[k];
            }
        }

        // Launches may be enqueued on different streams; a function's tiles can span
        // launches, so each launch waits for the previous one, and for the uploads
        // of the function tables it reads.
        // (A launch on the same stream is ordered already: a cross-stream wait on an
        // event of the same stream only adds latency.)
        {
            const LaunchSlot* newest = nullptr;
            for (const auto& o : ctx->slots)
                if (&o != &s && o.in_flight && (!newest || o.seq > newest->seq)) newest = &o;
            if (newest && newest->stream != stream) HIP_TRY(hipStreamWaitEvent(stream, newest->ev->done, 0));
        }
        for (Request* r : s.touched) {
            if (!r->uploaded) continue;
            const hipError_t q = hipEventQuery(r->uploaded);
            if (q == hipSuccess) {  // upload finished: nothing to wait for from now on
                quiet(hipEventDestroy(r->uploaded));
                r->uploaded = nullptr;
            } else {
                quiet(q);
                if (q != hipErrorNotReady) throw HipError{q, "hipEventQuery(upload)"};
                HIP_TRY(hipStreamWaitEvent(stream, r->uploaded, 0));
            }
        }
        // grids admitted while launches were in flight: their records are built in
        // this stream, before the stage kernel (and any graph) reads them
        for (Request* r : s.touched) {
            if (!r->grid || r->grid_packed) continue;
            DevFn* out = ctx->d_fns + r->slot_base;
            void* args[] = {&r->spec, &out};
            progress = std::max(progress, 1);
            HIP_TRY(hipLaunchKernel(pack_grid_kernel_ptr(), dim3((unsigned)((r->n + 255) / 256)), dim3(256), args, 0,
                                    stream));
            r->grid_packed = true;
        }
        EvSet& ev = *evp;
        s.ev = &ev;
        const uint64_t seq = ctx->launch_seq + 1;
        uint8_t* const hdesc_dev = s.h_block_dev + ctx->slot_res_bytes;
        LaunchDesc* hd = (LaunchDesc*)hdesc;
        std::memset(hdesc, 0, kDescBytes);
        hd->stage_bytes = kDescBytes + (uint64_t)s.n_fins * sizeof(Fin);
        hd->n_runs = s.n_runs;
        hd->runs_off = (uint32_t)(kDescBytes + (uint64_t)s.n_fins * sizeof(Fin));
        hd->fns = ctx->d_fns;
        hd->tiles = (const Tile*)(ddesc + kDescBytes + (uint64_t)ctx->fin_cap * sizeof(Fin));
        hd->partials = ctx->d_partials;
        hd->fins = (const Fin*)(ddesc + kDescBytes);
        hd->results = (DevResult*)ddesc - s.n_fins;
        hd->host_results = (DevResult*)hdesc_dev - s.n_fins;
        hd->counters = (uint32_t*)(ddesc + sizeof(LaunchDesc));
        hd->host_counters = (uint32_t*)(hdesc_dev + sizeof(LaunchDesc));
        hd->host_done = ctx->h_done_dev + 16 * (&s - ctx->slots);
        hd->seq = (uint32_t)seq;
        hd->abort_word = ctx->d_abort_word;
        hd->n_partials = ctx->max_partials;
        hd->n_fns = ctx->max_functions;
        for (int k = 0; k < kMaxKernels; ++k) {
            hd->tile_begin[k] = s.tile_begin[k];
            hd->tile_count[k] = s.tile_count[k];
        }
        hd->n_fins = s.n_fins;
        s.stream = stream;
        // a launch graph holds the built-in kernels only: with run-time families
        // registered, launches are enqueued directly
        s.graphed = ctx->use_graph && ctx->n_user == 0;
        ev.graphed = s.graphed;
        if (s.graphed) {
            if (!s.graph) capture_graph(ctx, s);
            HIP_TRY(hipEventRecord(ev.start, stream));
            progress = 2;  // a graph launch hands every kernel over at once
            HIP_TRY(hipGraphLaunch(s.graph, stream));
        } else {
            enqueue_kernels(ctx, s, stream, true, &progress);
        }
        // (ends the launch's timing intervals and orders launches on other
        // streams after this one; completion itself is read from the done word)
        HIP_TRY(hipEventRecord(ev.done, stream));
    } catch (const HipError&) {
        abandon_launch(ctx, s, stream, progress, req_undo, active_before);
        ctx->ev_free.push_back(evp);
        throw;
    }
    evp->pending = true;
    ctx->ev_pending.push_back(evp);
    s.in_flight = true;
    s.seq = ++ctx->launch_seq;
    log_msg(3, "launch %llu: %u tiles, %u results, %s", (unsigned long long)s.seq, s.n_tiles, s.n_fins,
            s.graphed ? "graph" : "direct");
    return true;
}

// Requests of a queue submitted before the abort call are taken out and
// collected in `out`; later ones stay (none of their work has been launched:
// the abort is carried out before anything else in the next step).
void take_aborted(mc_ctx* ctx, std::deque<Request*>& q, std::vector<Request*>& out)
{
    std::deque<Request*> keep;
    for (Request* r : q) {
        if (r->id < ctx->abort_below) out.push_back(r);
        else keep.push_back(r);
    }
    q.swap(keep);
}

// After mc_abort: let the launches in flight drain (their kernels stop at the
// next tile fetch), complete every request queued before the call with status
// MC_ERR_ABORTED, then clear the abort word so later work runs normally.
void finish_abort(mc_ctx* ctx)
{
    reap(ctx, 2);
    std::vector<Request*> cancel;
    take_aborted(ctx, ctx->active, cancel);
    take_aborted(ctx, ctx->pending, cancel);
    for (Request* r : cancel) complete_aborted(ctx, r);
    HIP_TRY(hipMemcpyAsync(ctx->d_abort_word, &ctx->h_words[0], sizeof(uint32_t), hipMemcpyHostToDevice,
                           ctx->upload_stream));
    HIP_TRY(hipStreamSynchronize(ctx->upload_stream));
    ctx->abort_requested = false;
}

// ---------------------------------------------------------------- resident engine

void res_publish(ResidentState& R)
{
    __atomic_store_n(R.ctl, R.pushed | (R.stopping ? kCtlStop : 0ull), __ATOMIC_RELEASE);
}

// Advance `acked` over the entries workgroups have read, in ring order.
void res_scan_acks(ResidentState& R)
{
    while (R.acked < R.pushed &&
           __atomic_load_n(&R.ack[R.acked & (kRingEntries - 1)], __ATOMIC_ACQUIRE) == R.acked + 1) {
        R.unread_tiles -= R.ring[R.acked & (kRingEntries - 1)].count;
        R.acked++;
    }
}

// Entries from `acked` on will never be read (abort, failed launch).
void res_drop_unread(ResidentState& R)
{
    R.acked = R.pushed;
    R.unread_tiles = 0;
}

// Whether the last launch has gone.  Every workgroup acknowledges what it read
// before it leaves, and the last one stores the exit word after that, so from
// here on the entries read are exactly [0, acked) (a stopping launch reads a
// prefix of the ring) and no workgroup touches the ring or a record again.
bool res_exited(mc_ctx* ctx)
{
    ResidentState& R = ctx->res;
    if (!R.live) return true;
    if (__atomic_load_n(R.exit_word, __ATOMIC_ACQUIRE) != R.epoch) return false;
    log_msg(2, "resident launch %u has left", R.epoch);
    R.live = false;
    R.stopping = false;
    R.flush = false;
    res_scan_acks(R);
    ctx->stats.bad_records = __atomic_load_n(R.exit_word + 1, __ATOMIC_RELAXED);  // (cumulative on the device)
    return true;
}

// Ask the running launch to end (its workgroups finish the entries below the
// count as it stands, then leave).  No entry is pushed until it has gone.
void res_request_stop(mc_ctx* ctx)
{
    ResidentState& R = ctx->res;
    if (!R.live || R.stopping) return;
    R.stopping = true;
    res_publish(R);
    log_msg(2, "resident launch %u: stop requested at ring entry %llu%s", R.epoch, (unsigned long long)R.pushed,
            R.flush ? " (record arena recycled)" : "");
}

// Start a launch if entries wait and none runs.
void res_launch(mc_ctx* ctx)
{
    ResidentState& R = ctx->res;
    if (!res_exited(ctx) || R.pushed == R.acked) return;
    uint32_t epoch = ++R.epoch;  // (a number whose launch failed is not reused)
    R.stage[0] = R.acked;
    R.stage[1] = R.pushed;
    R.stage[2] = R.grid;
    res_publish(R);
    bool enqueued = false;
    try {
        enqueued = true;
        HIP_TRY(hipMemcpyAsync(R.d_pos, R.stage, 2 * sizeof(uint64_t), hipMemcpyHostToDevice, R.stream));
        HIP_TRY(hipMemcpyAsync(R.d_running, &R.stage[2], sizeof(uint32_t), hipMemcpyHostToDevice, R.stream));
        ResidentDesc* d = R.d_desc;
        void* args[] = {&d, &epoch};
        if (R.user_kernel)
            HIP_TRY(hipModuleLaunchKernel(R.user_kernel, R.grid, 1, 1, kBlockThreads, 1, 1, 0, R.stream, args, nullptr));
        else
            HIP_TRY(hipLaunchKernel(resident_kernel_ptr(), dim3(R.grid), dim3(kBlockThreads), args, 0, R.stream));
    } catch (const HipError&) {
        // the staged start values are rewritten by the next attempt: let what
        // was enqueued finish first
        if (enqueued) quiet(hipStreamSynchronize(R.stream));
        throw;
    }
    R.live = true;
    ctx->stats.launches++;
    log_msg(2, "resident launch %u: %u workgroups, ring entries %llu..%llu", epoch, R.grid,
            (unsigned long long)R.acked, (unsigned long long)R.pushed);
}

// A record arena position for a new run.  Records are read through the
// scalar cache, which a kernel does not see invalidated while it runs, so a
// position may only be written again by a launch that started after every
// launch that read it: free means no run uses it and the launch the new run
// will be read in (the running one, or the next) has not read it.
bool res_alloc_rec(ResidentState& R, uint32_t* out)
{
    const uint32_t first_reader = R.live && !R.stopping ? R.epoch : R.epoch + 1;
    const uint32_t tries = R.live ? std::min(kArenaScan, R.n_arena) : R.n_arena;
    for (uint32_t k = 0; k < tries; ++k) {
        const uint32_t p = R.cursor;
        R.cursor = R.cursor + 1 == R.n_arena ? 0 : R.cursor + 1;
        if (!R.arena_busy[p] && R.arena_epoch[p] < first_reader) {
            *out = p;
            return true;
        }
    }
    return false;
}

bool res_room(const ResidentState& R)
{
    return !R.stopping && R.unread_tiles < R.backlog && R.pushed < R.acked + kRingEntries;
}

// Tiles of request r's next chunk (function state fs): one tile while the
// request's tiles not yet pushed do not fill the workgroups (its tiles spread
// over as many of them as possible), up to kChunkTiles as it has more (fewer
// entries for the host to write: the host writes one in tens of nanoseconds, a
// workgroup runs a tile in tens of microseconds, so a saturated GPU needs
// entries of several tiles).
uint32_t res_chunk_tiles(const ResidentState& R, const Request* r, const FnState& fs)
{
    const uint32_t left = fs.n_tiles - fs.next_tile;
    const uint64_t per_wg = (r->tiles_total - r->tiles_launched) / R.grid;
    return std::min(std::min(left, kChunkTiles), (uint32_t)std::max<uint64_t>(1, per_wg));
}

// Push request r's next chunk into the ring (not yet published).  The first
// chunk of a run takes a token and an arena position and carries the upload
// flag.  Returns false if nothing was pushed.
bool res_push_chunk(mc_ctx* ctx, Request* r)
{
    ResidentState& R = ctx->res;
    if (!has_work(r) || !res_room(R) || r->partials_pending) return false;
    const bool in_order = r->order_pos < r->order.size();
    const uint32_t fi = in_order ? r->order[r->order_pos] : r->redo[r->redo_pos];
    FnState& fs = r->st[fi];
    // a run starts at tile 0, or, for a restored function, at the first tile
    // its snapshot had not run
    const bool first = fs.next_tile == 0 || fs.token == 0;
    if (first) {
        uint32_t rec = 0;
        if (R.flush || !res_alloc_rec(R, &rec)) {
            R.flush = true;
            return false;
        }
        if (++R.next_token == 0) ++R.next_token;
        fs.token = R.next_token;
        fs.rec = rec;
        R.arena_busy[rec] = 1;
        R.runs.push_back(ResRun{r, fi, fs.slot, fs.token, rec});
    }
    const uint32_t count = res_chunk_tiles(R, r, fs);
    R.ring[R.pushed & (kRingEntries - 1)] =
        Chunk{fs.slot, fs.rec, fs.next_tile, count, (uint32_t)fs.part0, fs.n_tiles, fs.token,
              fs.seg_log2 | (first ? kChunkUpload << 8 : 0u)};
    R.pushed++;
    R.unread_tiles += count;
    R.tiles_waiting -= std::min<uint64_t>(R.tiles_waiting, count);
    fs.next_tile += count;
    fs.needs_upload = false;
    r->tiles_launched += count;
    r->work_left = std::max(0.0, r->work_left - fs.tile_cost * (double)count);
    if (fs.f64) ctx->stats.tiles64 += count;
    else ctx->stats.tiles32 += count;
    if (fs.next_tile == fs.n_tiles) {
        if (in_order) r->order_pos++;
        else r->redo_pos++;
    }
    return true;
}

// Fill the ring up to the backlog by the scheduling policy: FIFO from the
// oldest request, SRPT from the request with the least work left (the list is
// re-sorted only when admission or a promotion may have changed the order:
// pushing from the first request only makes it smaller), FAIR one chunk per
// request in turn, each fill starting where the previous one stopped.
void res_feed(mc_ctx* ctx)
{
    ResidentState& R = ctx->res;
    res_scan_acks(R);
    if (!res_room(R) || ctx->active.empty()) return;
    const uint64_t before = R.pushed;
    bool exhausted = false;
    if (ctx->policy == MC_SCHED_SRPT && R.active_dirty) {
        std::stable_sort(ctx->active.begin(), ctx->active.end(),
                         [](const Request* a, const Request* b) { return a->work_left < b->work_left; });
        R.active_dirty = false;
    }
    if (ctx->policy == MC_SCHED_FAIR) {
        // deficit round robin by tiles: each visit credits a request with
        // kChunkTiles tiles and it pushes chunks while its credit covers the
        // next one, so requests cut into large chunks get no larger share
        const size_t n = ctx->active.size();
        size_t k = R.fair_pos % n, idle = 0;
        while (idle < n && res_room(R) && !R.flush) {
            Request* r = ctx->active[k];
            bool pushed = false;
            if (has_work(r)) {
                r->fair_credit = std::min(r->fair_credit + kChunkTiles, 2 * kChunkTiles);
                while (has_work(r) && res_room(R)) {
                    const bool in_order = r->order_pos < r->order.size();
                    const uint32_t fi = in_order ? r->order[r->order_pos] : r->redo[r->redo_pos];
                    const uint32_t need = res_chunk_tiles(R, r, r->st[fi]);
                    if (need > r->fair_credit || !res_push_chunk(ctx, r)) break;
                    r->fair_credit -= need;
                    pushed = true;
                }
            }
            idle = pushed ? 0 : idle + 1;
            if (!has_work(r)) exhausted = true;
            k = k + 1 == n ? 0 : k + 1;
        }
        R.fair_pos = k;
    } else {
        for (Request* r : ctx->active) {
            while (res_push_chunk(ctx, r)) {
            }
            if (!has_work(r)) exhausted = true;
            if (!res_room(R) || R.flush) break;
        }
    }
    if (exhausted) {
        std::deque<Request*> keep;
        for (Request* r : ctx->active)
            if (has_work(r)) keep.push_back(r);
        ctx->active.swap(keep);
    }
    if (R.pushed != before) res_publish(R);
    // arena positions of the running launch are exhausted: end it, so that
    // the next one may reuse them
    if (R.flush) res_request_stop(ctx);
}

// Results of runs whose done word shows their token.
void res_reap(mc_ctx* ctx)
{
    ResidentState& R = ctx->res;
    size_t w = 0;
    const size_t n = R.runs.size();
    for (size_t i = 0; i < n; ++i) {
        const ResRun run = R.runs[i];
        if (__atomic_load_n(&R.done[run.slot], __ATOMIC_ACQUIRE) != run.token) {
            R.runs[w++] = run;
            continue;
        }
        DevResult res;
        std::memcpy(&res, &R.results[run.slot], sizeof res);
        R.arena_busy[run.rec] = 0;
        R.arena_epoch[run.rec] = R.epoch;
        ctx->stats.functions++;
        ctx->stats.samples += res.n;
        complete_function(ctx, run.req, run.index, res, false);
    }
    R.runs.resize(w);
}

void res_fail(mc_ctx* ctx);

// Wait until the last launch has gone.  The kernel leaves by itself (a
// stopping launch within a chunk per workgroup, an idle one within its poll
// bound); a stream that reports an error, or that is idle while the exit word
// never came, is an error.
void res_wait_exit(mc_ctx* ctx)
{
    ResidentState& R = ctx->res;
    for (uint64_t i = 0; !res_exited(ctx); ++i) {
        if (i < 4096) continue;
        if (i < 65536) {
            sched_yield();
            continue;
        }
        if ((i & 255) == 0) {
            const hipError_t q = hipStreamQuery(R.stream);
            quiet(q);
            if (q != hipErrorNotReady) {
                if (res_exited(ctx)) return;
                res_fail(ctx);
                if (q != hipSuccess) throw HipError{q, "hipStreamQuery(resident launch)"};
                throw HipError{hipErrorUnknown, "resident launch finished without its exit word"};
            }
        }
        struct timespec ts{0, 20000};
        nanosleep(&ts, nullptr);
    }
}

// The resident launch failed (an error from its stream, or it never stored its
// exit word): every run in the ring is lost and its request completes with
// MC_ERR_HIP; with the stream idle nothing refers to their slots any more.
void res_fail(mc_ctx* ctx)
{
    ResidentState& R = ctx->res;
    for (const ResRun& run : R.runs) {
        Request* r = run.req;
        R.arena_busy[run.rec] = 0;
        R.arena_epoch[run.rec] = R.epoch;
        if (r->lost) continue;
        r->lost = true;
        r->order_pos = (uint32_t)r->order.size();
        r->redo_pos = (uint32_t)r->redo.size();
        r->tiles_launched = r->tiles_total;
        r->work_left = 0.0;
    }
    R.runs.clear();
    std::deque<Request*> keep;
    for (Request* r : ctx->active)
        if (!r->lost) keep.push_back(r);
    ctx->active.swap(keep);
    R.live = false;
    R.stopping = false;
    R.flush = false;
    res_drop_unread(R);
    R.tiles_waiting = 0;
    for (Request* r : ctx->active) R.tiles_waiting += r->tiles_total - r->tiles_launched;
    __atomic_store_n(R.ctl, R.pushed, __ATOMIC_RELEASE);
    // the lost runs' tile counters would mislead the next runs in their slots
    // (after a stream error these calls fail too, and so does every later launch)
    quiet(hipMemsetAsync(R.d_tiles_done, 0, (size_t)ctx->max_functions * sizeof(uint32_t), R.stream));
    quiet(hipStreamSynchronize(R.stream));
}

// After mc_abort on a resident context: the launch has been asked to stop;
// once it has gone, results that came in complete normally, every other
// request submitted before the call completes as aborted, the unread entries
// are dropped and the slot counters the cancelled runs leave behind are
// cleared.  Requests submitted later have nothing in the ring yet (the ring is
// fed only after the abort is carried out) and stay queued.
void res_finish_abort(mc_ctx* ctx)
{
    ResidentState& R = ctx->res;
    res_request_stop(ctx);
    res_wait_exit(ctx);
    res_reap(ctx);
    std::vector<Request*> cancel;
    for (const ResRun& run : R.runs) {
        R.arena_busy[run.rec] = 0;
        R.arena_epoch[run.rec] = R.epoch;
        cancel.push_back(run.req);
    }
    R.runs.clear();
    take_aborted(ctx, ctx->active, cancel);
    take_aborted(ctx, ctx->pending, cancel);
    for (Request* r : cancel)
        if (r->fns_done < r->count()) complete_aborted(ctx, r);  // (a request can be listed twice)
    res_drop_unread(R);
    R.tiles_waiting = 0;
    for (Request* r : ctx->active) R.tiles_waiting += r->tiles_total - r->tiles_launched;
    __atomic_store_n(R.ctl, R.pushed, __ATOMIC_RELEASE);
    HIP_TRY(hipMemsetAsync(R.d_tiles_done, 0, (size_t)ctx->max_functions * sizeof(uint32_t), R.stream));
    HIP_TRY(hipStreamSynchronize(R.stream));
    ctx->abort_requested = false;
}

// Restored requests: their saved partials, and their functions' tile counts
// (a run's finalizer is the workgroup that counts its last tile), go to the
// device on the resident stream while no launch runs -- a running one is asked
// to stop first --, so the next launch, enqueued after the copies, sees them.
// Until then none of the requests' chunks is pushed.
void res_upload_restored(mc_ctx* ctx)
{
    ResidentState& R = ctx->res;
    bool any = false;
    for (const Request* r : ctx->active) any = any || r->partials_pending;
    if (!any) return;
    if (!res_exited(ctx)) {
        res_request_stop(ctx);
        return;
    }
    for (Request* r : ctx->active) {
        if (!r->partials_pending) continue;
        HIP_TRY(hipMemcpyAsync(ctx->d_partials + r->part_base, r->staged.data(), r->part_count * sizeof(Partial),
                               hipMemcpyHostToDevice, R.stream));
        HIP_TRY(hipMemcpyAsync(R.d_tiles_done + r->slot_base, r->staged_counts.data(), r->count() * sizeof(uint32_t),
                               hipMemcpyHostToDevice, R.stream));
        r->partials_pending = false;
        log_msg(3, "request %llu: saved partials copied to the device", (unsigned long long)r->id);
    }
}

// mc_cancel of an admitted request in a resident context (its work already
// dropped).  Its slots go back to the pool, and every slot of the pool must
// hold a tile count of zero: a slot's counter is non-zero while a run in it is
// open, and, for a restored request whose saved counts were copied to the
// device, from that copy until the function's run finalizes.  In either case
// the launch is stopped (it runs every entry below its count, then leaves) and
// the results that came in are collected (and dropped); the request's entries
// it did not read (only after an idle stop) are taken out of the ring, the
// others keeping their order, while no kernel runs; its open runs give back
// their arena positions, and its slots' tile counters are cleared.  Then it
// completes as aborted.  If clearing the counters fails, it completes all the
// same but keeps its slots (their counters are unknown), and the error is
// passed on.
void res_cancel(mc_ctx* ctx, Request* r)
{
    ResidentState& R = ctx->res;
    bool open = false;
    for (const ResRun& run : R.runs) open = open || run.req == r;
    bool counted = false;  // saved counts on the device of functions without their result
    if (!r->partials_pending)
        for (size_t i = 0; i < r->staged_counts.size(); ++i) counted = counted || (r->staged_counts[i] && !r->st[i].done);
    if (open || counted) {
        res_request_stop(ctx);
        res_wait_exit(ctx);
        res_reap(ctx);
        uint64_t w = R.acked;
        for (uint64_t e = R.acked; e < R.pushed; ++e) {
            const Chunk c = R.ring[e & (kRingEntries - 1)];
            const bool mine = c.fn >= r->slot_base && c.fn - r->slot_base < r->count() &&
                              c.token == r->st[c.fn - r->slot_base].token;
            if (mine) {
                R.unread_tiles -= c.count;
                continue;
            }
            R.ring[w++ & (kRingEntries - 1)] = c;
        }
        R.pushed = w;
        size_t k = 0;
        bool runs_left = false;
        for (const ResRun& run : R.runs) {
            if (run.req != r) {
                R.runs[k++] = run;
                continue;
            }
            R.arena_busy[run.rec] = 0;
            R.arena_epoch[run.rec] = R.epoch;
            runs_left = true;
        }
        R.runs.resize(k);
        if (runs_left || counted) {
            try {
                HIP_TRY(hipMemsetAsync(R.d_tiles_done + r->slot_base, 0, r->count() * sizeof(uint32_t), R.stream));
                HIP_TRY(hipStreamSynchronize(R.stream));
            } catch (const HipError&) {
                r->admitted = false;  // (its slots are not released)
                complete_aborted(ctx, r);
                throw;
            }
        }
    }
    complete_aborted(ctx, r);
}

// One step of a resident context: collect results, admit, feed the ring and
// (re)launch the kernel if entries wait and it has gone.
void res_step(mc_ctx* ctx)
{
    ResidentState& R = ctx->res;
    res_exited(ctx);
    res_reap(ctx);
    if (ctx->abort_requested) res_finish_abort(ctx);
    admit(ctx);
    res_upload_restored(ctx);
    res_feed(ctx);
    if (!R.live) res_launch(ctx);
}

// Whether the resident launch is known to have failed; checks the stream.
bool res_stream_failed(mc_ctx* ctx)
{
    ResidentState& R = ctx->res;
    if (!R.live) return false;
    const hipError_t q = hipStreamQuery(R.stream);
    quiet(q);
    if (q == hipErrorNotReady) return false;
    if (res_exited(ctx)) return false;
    return true;  // an error, or idle without the exit word
}

void destroy_device(mc_ctx* ctx)
{
    ResidentState& R = ctx->res;
    if (R.stream) quiet(hipStreamDestroy(R.stream));
    R.stream = nullptr;
    if (R.user_module) quiet(hipModuleUnload(R.user_module));
    R.user_module = nullptr;
    R.user_kernel = nullptr;
    if (R.h_block) quiet(hipHostFree(R.h_block));
    R.h_block = nullptr;
    for (auto& s : ctx->slots) {
        if (s.graph) quiet(hipGraphExecDestroy(s.graph));
        if (s.h_block) quiet(hipHostFree(s.h_block));
        s = LaunchSlot{};
    }
    if (ctx->upload_stream) quiet(hipStreamDestroy(ctx->upload_stream));
    ctx->upload_stream = nullptr;
    for (uint32_t u = 0; u < ctx->n_user; ++u)
        if (ctx->user[u].module) quiet(hipModuleUnload(ctx->user[u].module));
    ctx->n_user = 0;
    for (auto& e : ctx->ev_pool)
        for (hipEvent_t x : {e->start, e->mid, e->main, e->done})
            if (x) quiet(hipEventDestroy(x));
    ctx->ev_pool.clear();
    ctx->ev_free.clear();
    ctx->ev_pending.clear();
    if (ctx->h_fns) quiet(hipHostFree(ctx->h_fns));
    ctx->h_fns = nullptr;
    if (ctx->h_words) quiet(hipHostFree(ctx->h_words));
    if (ctx->h_done) quiet(hipHostFree(ctx->h_done));
    ctx->h_done = nullptr;
    if (ctx->owns_memory && ctx->mem_base) quiet(hipFree(ctx->mem_base));
    ctx->h_words = nullptr;
    ctx->mem_base = nullptr;
}

// Tile size before any tuning: 4 segments per workgroup (one per wave) from
// d = 3 on; at d = 1 and 2 a segment is so short that the per-tile fetch,
// barriers and tree would dominate (measured at d = 1: 0.45 of the VALU
// roofline with one segment per wave, 0.65 with four), so such tiles hold 4
// and 2 segments per wave.
void default_tuning(mc_ctx* ctx)
{
    for (int p = 0; p < 2; ++p)
        for (int f = 0; f < kNumFamilies; ++f)
            for (int d = 0; d < kMaxDim; ++d) ctx->seg_log2[p][f][d] = d == 0 ? 2 : d == 1 ? 1 : 0;
}

// Device state of a resident context: its stream, the pinned host block
//   [ring | acknowledgements | control word | exit word | start values | results | done words]
// and, in device memory, the descriptor, counters, per-slot words, ready words
// (zeroed: tokens start at 1) and the record arena.
void create_resident(mc_ctx* ctx, const Layout& L, uint8_t* base)
{
    ResidentState& R = ctx->res;
    const mc_config& cfg = ctx->cfg;
    int occ = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, resident_kernel_ptr(), kBlockThreads, 0));
    R.grid = (uint32_t)ctx->num_cus * (cfg.blocks_per_cu ? cfg.blocks_per_cu : (uint32_t)std::max(1, occ));
    // by default two tiles per workgroup wait unread: enough for the host to
    // refill before the workgroups run dry, little for a new request to wait behind
    R.backlog = cfg.max_tiles_per_run ? cfg.max_tiles_per_run : 2ull * R.grid;
    R.n_arena = L.n_arena;
    R.arena_epoch.assign(R.n_arena, 0u);
    R.arena_busy.assign(R.n_arena, 0u);
    const uint64_t ring_off = 0;
    const uint64_t ack_off = ring_off + (uint64_t)kRingEntries * sizeof(Chunk);
    const uint64_t ctl_off = ack_off + (uint64_t)kRingEntries * sizeof(uint64_t);
    const uint64_t exit_off = ctl_off + 64;
    const uint64_t stage_off = exit_off + 64;
    const uint64_t res_off = stage_off + 256;
    const uint64_t done_off = res_off + (uint64_t)ctx->max_functions * sizeof(DevResult);
    const uint64_t bytes = done_off + (uint64_t)ctx->max_functions * sizeof(uint32_t);
    HIP_TRY(hipHostMalloc((void**)&R.h_block, bytes, hipHostMallocMapped | hipHostMallocCoherent));
    HIP_TRY(hipHostGetDevicePointer((void**)&R.h_block_dev, R.h_block, 0));
    std::memset(R.h_block, 0, bytes);
    R.ring = (Chunk*)(R.h_block + ring_off);
    R.ack = (uint64_t*)(R.h_block + ack_off);
    R.ctl = (uint64_t*)(R.h_block + ctl_off);
    R.exit_word = (uint32_t*)(R.h_block + exit_off);
    R.stage = (uint64_t*)(R.h_block + stage_off);
    R.results = (DevResult*)(R.h_block + res_off);
    R.done = (uint32_t*)(R.h_block + done_off);
    HIP_TRY(hipStreamCreateWithFlags(&R.stream, hipStreamNonBlocking));
    R.d_desc = (ResidentDesc*)(base + L.res_desc);
    R.d_pos = (uint64_t*)(base + L.res_desc + 256);
    R.d_running = (uint32_t*)(base + L.res_desc + 256 + 16);
    R.d_bad = (uint32_t*)(base + L.res_desc + 256 + 20);
    R.d_tiles_done = (uint32_t*)(base + L.res_tiles_done);
    static_assert(sizeof(ResidentDesc) <= 256, "resident descriptor size");
    ResidentDesc D{};
    uint8_t* hb = R.h_block_dev;
    D.ring = (const Chunk*)(hb + ring_off);
    D.ack = (uint64_t*)(hb + ack_off);
    D.host_ctl = (const uint64_t*)(hb + ctl_off);
    D.host_exit = (uint32_t*)(hb + exit_off);
    D.host_results = (DevResult*)(hb + res_off);
    D.host_done = (uint32_t*)(hb + done_off);
    D.mirror = ctx->h_fns_dev;
    D.arena = (DevFn*)(base + L.res_arena);
    D.partials = ctx->d_partials;
    D.pos = R.d_pos;
    D.running = R.d_running;
    D.tiles_done = R.d_tiles_done;
    D.ready = (uint32_t*)(base + L.res_ready);
    D.slot_err = (uint32_t*)(base + L.res_slot_err);
    D.bad_records = R.d_bad;
    D.n_partials = ctx->max_partials;
    D.n_fns = ctx->max_functions;
    D.n_arena = R.n_arena;
    D.ring_mask = kRingEntries - 1;
    D.idle_polls = kIdlePolls;
    D.ready_polls = kReadyPolls;
    D.leader_every = kLeaderEvery;
    // the descriptor goes up through the start-value block (256 bytes, unused
    // until the first launch); the words after it are zeroed
    std::memcpy(R.stage, &D, sizeof D);
    HIP_TRY(hipMemcpyAsync(R.d_desc, R.stage, sizeof D, hipMemcpyHostToDevice, R.stream));
    HIP_TRY(hipMemsetAsync(base + L.res_desc + 256, 0, L.res_arena - (L.res_desc + 256), R.stream));
    HIP_TRY(hipStreamSynchronize(R.stream));
    std::memset(R.stage, 0, 256);
}

// mc_results on a resident context.  A blocking wait steps the context (which
// keeps the ring fed and relaunches the kernel when it has gone), spinning,
// then yielding, then sleeping in short steps, and checks the launch's stream
// now and then: an error, or an idle stream whose launch never stored its exit
// word, fails the runs in the ring instead of waiting for them.
mc_status res_results(mc_ctx* ctx, std::unordered_map<uint64_t, std::unique_ptr<Request>>::iterator it,
                      mc_result* out, size_t n, int blocking)
{
    Request* r = it->second.get();
    const uint64_t id = r->id;
    try {
        HIP_TRY(hipSetDevice(ctx->device));
        for (uint64_t i = 0; r->fns_done < r->count(); ++i) {
            if (r->lost) {
                free_request_resources(ctx, r);
                ctx->requests.erase(it);
                return fail(ctx, MC_ERR_HIP, "request %llu cannot complete: the resident launch failed",
                            (unsigned long long)id);
            }
            res_step(ctx);
            if (r->fns_done == r->count() || r->lost) continue;
            if (!blocking) return MC_NOT_READY;
            if (i < 2048) continue;
            if (i < 16384) {
                sched_yield();
                continue;
            }
            if ((i & 255) == 0 && res_stream_failed(ctx)) {
                res_fail(ctx);
                continue;
            }
            struct timespec ts{0, 20000};
            nanosleep(&ts, nullptr);
        }
    } catch (const HipError& e) {
        return fail_hip(ctx, e);
    }
    std::memcpy(out, r->results.data(), n * sizeof(mc_result));
    const bool aborted = r->aborted;
    ctx->requests.erase(it);
    return aborted ? MC_ERR_ABORTED : MC_OK;
}

}  // namespace

// ====================================================================== C ABI

extern "C" {

mc_status mc_config_init(mc_config* cfg)
{
    if (!cfg) return fail(nullptr, MC_ERR_INVALID_ARG, "cfg is NULL");
    std::memset(cfg, 0, sizeof(*cfg));
    return MC_OK;
}

mc_status mc_workspace_size(const mc_config* cfg, uint64_t* bytes)
{
    if (!cfg || !bytes) return fail(nullptr, MC_ERR_INVALID_ARG, "NULL argument");
    uint32_t mf, tc, fc;
    uint64_t mp;
    resolve_capacities(*cfg, &mf, &mp, &tc, &fc);
    *bytes = compute_layout(mf, mp, tc, fc, (cfg->flags & MC_RESIDENT) != 0).total;
    return MC_OK;
}

mc_status mc_create(const mc_config* cfg_in, mc_ctx** out)
{
    if (!out) return fail(nullptr, MC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    mc_config cfg{};
    if (cfg_in) cfg = *cfg_in;
    std::unique_ptr<mc_ctx> ctx(new mc_ctx());
    ctx->cfg = cfg;
    ctx->validate_only = (cfg.flags & MC_VALIDATE_ONLY) != 0;
    ctx->use_graph = (cfg.flags & MC_NO_GRAPH) == 0;
    ctx->promote = (cfg.flags & MC_NO_PROMOTE) == 0;
    ctx->res.on = (cfg.flags & MC_RESIDENT) != 0;
    ctx->device = cfg.device;
    if (cfg.policy > MC_SCHED_SRPT) return fail(nullptr, MC_ERR_INVALID_ARG, "unknown policy %u", cfg.policy);
    // tiles, finalize records and partial indices are 32-bit; the pinned mirror holds 1 KiB per slot
    if (cfg.max_partials > 0xFFFFFFFFull)
        return fail(nullptr, MC_ERR_INVALID_ARG, "max_partials above 2^32 - 1");
    if (cfg.max_functions > (1u << 24)) return fail(nullptr, MC_ERR_INVALID_ARG, "max_functions above 2^24");
    if (cfg.max_tiles_per_run > (1u << 28)) return fail(nullptr, MC_ERR_INVALID_ARG, "max_tiles_per_run above 2^28");
    ctx->policy = cfg.policy;
    default_tuning(ctx.get());
    resolve_capacities(cfg, &ctx->max_functions, &ctx->max_partials, &ctx->tile_cap, &ctx->fin_cap);
    ctx->fn_alloc.reset(ctx->max_functions);
    ctx->part_alloc.reset(ctx->max_partials);
    arm_log_level();
    if (ctx->validate_only) {
        *out = ctx.release();
        return MC_OK;
    }
    arm_fault_injection();
    try {
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= cfg.device || cfg.device < 0)
            return fail(nullptr, MC_ERR_NO_DEVICE, "no HIP device %d (found %d)", cfg.device, ndev);
        HIP_TRY(hipSetDevice(cfg.device));
        hipDeviceProp_t prop;
        HIP_TRY(hipGetDeviceProperties(&prop, cfg.device));
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
            return fail(nullptr, MC_ERR_NO_DEVICE, "device %d is %s; this library is built for gfx950", cfg.device,
                        prop.gcnArchName);
        ctx->num_cus = prop.multiProcessorCount;
        ctx->device_name = prop.gcnArchName;
        HIP_TRY(scratch_address(cfg.device, &ctx->scratch));
        int occ32 = 0, occ64 = 0;
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ32, batched_kernel_ptr(false), kBlockThreads, 0));
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ64, batched_kernel_ptr(true), kBlockThreads, 0));
        ctx->blocks_per_cu32 = cfg.blocks_per_cu ? cfg.blocks_per_cu : (uint32_t)std::max(1, occ32);
        ctx->blocks_per_cu64 = (uint32_t)std::max(1, occ64);

        Layout L = compute_layout(ctx->max_functions, ctx->max_partials, ctx->tile_cap, ctx->fin_cap, ctx->res.on);
        ctx->slot_res_bytes = L.slot_res_bytes;
        ctx->slot_bytes = L.slot_bytes;
        if (cfg.mem_budget_bytes && L.total > cfg.mem_budget_bytes)
            return fail(nullptr, MC_ERR_OUT_OF_MEMORY, "context needs %llu device bytes, budget is %llu",
                        (unsigned long long)L.total, (unsigned long long)cfg.mem_budget_bytes);
        if (cfg.workspace) {
            if (cfg.workspace_bytes < L.total)
                return fail(nullptr, MC_ERR_INVALID_ARG, "workspace of %llu bytes is smaller than the %llu needed",
                            (unsigned long long)cfg.workspace_bytes, (unsigned long long)L.total);
            if (((uintptr_t)cfg.workspace & 255u) != 0)
                return fail(nullptr, MC_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
            ctx->owns_memory = false;
            ctx->mem_base = cfg.workspace;
        } else {
            const hipError_t e = fault_due() ? hipErrorOutOfMemory : hipMalloc(&ctx->mem_base, L.total);
            if (e != hipSuccess) {
                quiet(e);
                ctx->mem_base = nullptr;
                mc_status st = fail(nullptr, MC_ERR_OUT_OF_MEMORY, "hipMalloc of %llu bytes failed",
                                    (unsigned long long)L.total);
                destroy_device(ctx.get());
                return st;
            }
        }
        ctx->mem_bytes = L.total;
        uint8_t* base = (uint8_t*)ctx->mem_base;
        ctx->d_fns = ctx->res.on ? nullptr : (DevFn*)(base + L.fns);
        ctx->d_partials = (Partial*)(base + L.partials);
        for (int i = 0; i < (ctx->res.on ? 0 : kLaunchSlots); ++i) {
            LaunchSlot& s = ctx->slots[i];
            s.d_block = base + L.slots + (uint64_t)i * L.slot_bytes;
            s.d_desc = (LaunchDesc*)(s.d_block + L.slot_res_bytes);
            // fine-grained: kernels read the staged launch and write results into it
            HIP_TRY(hipHostMalloc((void**)&s.h_block, L.slot_bytes, hipHostMallocMapped | hipHostMallocCoherent));
            HIP_TRY(hipHostGetDevicePointer((void**)&s.h_block_dev, s.h_block, 0));
        }
        HIP_TRY(hipHostMalloc((void**)&ctx->h_fns, (size_t)ctx->max_functions * sizeof(DevFn),
                              hipHostMallocMapped | hipHostMallocCoherent));
        HIP_TRY(hipHostGetDevicePointer((void**)&ctx->h_fns_dev, ctx->h_fns, 0));
        HIP_TRY(hipHostMalloc((void**)&ctx->h_done, kLaunchSlots * 16 * sizeof(uint32_t),
                              hipHostMallocMapped | hipHostMallocCoherent));
        HIP_TRY(hipHostGetDevicePointer((void**)&ctx->h_done_dev, ctx->h_done, 0));
        std::memset(ctx->h_done, 0, kLaunchSlots * 16 * sizeof(uint32_t));
        HIP_TRY(hipStreamCreateWithFlags(&ctx->upload_stream, hipStreamNonBlocking));
        HIP_TRY(hipHostMalloc((void**)&ctx->h_words, 2 * sizeof(uint32_t), hipHostMallocDefault));
        ctx->h_words[0] = 0u;
        ctx->h_words[1] = 1u;
        ctx->d_abort_word = (uint32_t*)(base + L.abort_word);
        HIP_TRY(hipMemcpyAsync(ctx->d_abort_word, &ctx->h_words[0], sizeof(uint32_t), hipMemcpyHostToDevice,
                               ctx->upload_stream));
        HIP_TRY(hipStreamSynchronize(ctx->upload_stream));
        if (ctx->res.on) create_resident(ctx.get(), L, base);
    } catch (const HipError& e) {
        mc_status st = fail_hip(nullptr, e);
        destroy_device(ctx.get());
        return st;
    }
    log_msg(2, "context on device %d (%s, %d CUs): %u function slots, %llu partials, %llu device bytes%s", ctx->device,
            ctx->device_name.c_str(), ctx->num_cus, ctx->max_functions, (unsigned long long)ctx->max_partials,
            (unsigned long long)ctx->mem_bytes, ctx->res.on ? ", resident" : "");
    *out = ctx.release();
    return MC_OK;
}

mc_status mc_destroy(mc_ctx* ctx)
{
    if (!ctx) return MC_OK;
    if (!ctx->validate_only) {
        quiet(hipSetDevice(ctx->device));
        for (auto& s : ctx->slots)
            if (s.in_flight && s.ev) quiet(hipEventSynchronize(s.ev->done));
        if (ctx->res.on && ctx->res.stream) {
            // ask a running launch to leave and wait for it (it leaves within a
            // chunk per workgroup once it has seen the stop bit)
            res_request_stop(ctx);
            quiet(hipStreamSynchronize(ctx->res.stream));
        }
    }
    if (!ctx->validate_only) {
        // requests still in the context may hold the event of their upload
        for (auto& kv : ctx->requests)
            if (kv.second->uploaded) {
                quiet(hipEventDestroy(kv.second->uploaded));
                kv.second->uploaded = nullptr;
            }
        destroy_device(ctx);
    }
    delete ctx;
    return MC_OK;
}

namespace {

// Largest phase, in revolutions, that the FP32 evaluation of Eq. (1) carries:
// theta = f0 + sum_j kappa_j t_j with f0 in [0, 1), t_j in [1, 2) and
// kappa_j = k_j w_j / 2 pi, so |theta| < 1 + 2 sum_j |kappa_j|.  Its FP32
// rounding grows with it (measured: about 2.2e-7 * theta standard errors on
// the estimate, whatever N), so beyond kFp32MaxPhaseRev (about 1e-3 SE) the
// function is evaluated in FP64 instead.  0 for the other families.
constexpr double kFp32MaxPhaseRev = 4096.0;

double fp32_phase_bound(const mc_function& f)
{
    if (f.family != MC_FAMILY_HARMONIC) return 0.0;
    double th = 1.0;
    for (uint32_t j = 0; j < f.dim && j < (uint32_t)MC_MAX_DIM; ++j)
        th += 2.0 * std::fabs(f.params[MC_PARAM_V0 + j] * (f.hi[j] - f.lo[j])) / kPackTwoPi;
    return th;
}

// The product polynomial and run-time families see the sample point in FP32
// absolute coordinates, x_j = fma(w_j, u_j, lo_j) with lo_j and w_j rounded to
// float: a shift common to all samples of about 2^-25 max(|lo_j|, |hi_j|),
// which against the box width biases the estimate by about
// 2^-25 sqrt(12) K sqrt(N) standard errors, K = max_j max(|lo_j|, |hi_j|) / w_j
// (measured on the GPU: K = 100, N = 1e6, a factor with its root in the box:
// 1.1e-2 SE, against 1.0e-2 predicted).  Where that exceeds 0.0025 SE, i.e.
// K sqrt(N) > kFp32MaxOffsetRootN, the function is evaluated in FP64 instead.
// 0 for the families evaluated in local coordinates.
constexpr double kFp32MaxOffsetRootN = 24200.0;

double fp32_offset_ratio(const mc_function& f)
{
    if (f.family <= (uint32_t)MC_FAMILY_GAUSSIAN) return 0.0;
    double k = 0.0;
    for (uint32_t j = 0; j < f.dim && j < (uint32_t)MC_MAX_DIM; ++j)
        k = std::max(k, std::max(std::fabs(f.lo[j]), std::fabs(f.hi[j])) / (f.hi[j] - f.lo[j]));
    return k;
}

// From this many samples on the check after an FP32 run (fp32_unresolved:
// sigma / rms below 400 * 2^-24 * sqrt(N), a bound above 1 + 1/N here) re-runs
// every function in FP64, since sigma / rms never exceeds that; such functions
// go to FP64 at submit instead, with the same result and no FP32 pass.
constexpr double kFp32MaxSamples = 1.8e9;

// Whether FP32 evaluation of f can meet 0.01 SE at all (checked at submit).
bool fp32_hopeless(const mc_function& f)
{
    return (double)f.n_samples >= kFp32MaxSamples || fp32_phase_bound(f) > kFp32MaxPhaseRev ||
           fp32_offset_ratio(f) * std::sqrt((double)f.n_samples) > kFp32MaxOffsetRootN;
}

// Scheduling state of function i, common to tables and grids; `f64`: evaluated
// by the FP64 kernels.
void init_fn_state(mc_ctx* ctx, Request* r, size_t i, const mc_function& f, bool f64)
{
    struct {
        uint32_t family, dim, n_segments;
        uint64_t n_samples;
    } d{f.family, f.dim, (uint32_t)(((f.n_samples + 3) / 4 + kSegQuads - 1) / kSegQuads), f.n_samples};
    FnState& fs = r->st[i];
    // run-time families take the harmonic family's tile size
    const uint32_t tf = d.family < (uint32_t)kNumFamilies ? d.family : (uint32_t)MC_FAMILY_HARMONIC;
    uint32_t L = ctx->seg_log2[f64 ? 1 : 0][tf][d.dim - 1];
    // no point in tiles larger than the function; very large functions take
    // larger tiles so their partials stay within kTargetTilesPerFn (results do
    // not depend on the tile size)
    while (L > 0 && ((uint32_t)kBlockWaves << (L - 1)) >= d.n_segments) --L;
    while (L < (uint32_t)kMaxSegLog2 && tiles_for(d.n_segments, L) > kTargetTilesPerFn) ++L;
    fs.seg_log2 = L;
    fs.n_tiles = tiles_for(d.n_segments, L);
    fs.next_tile = 0;
    fs.f64 = f64;
    fs.needs_upload = false;
    fs.token = 0;
    fs.rec = 0;
    fs.done = false;
    fs.tile_cost = sample_cost(d.family, d.dim, f64 ? MC_PREC_FP64 : MC_PREC_FP32_EVAL) *
                   (double)std::min<uint64_t>(d.n_samples, (uint64_t)kSegSamples * ((uint64_t)kBlockWaves << L));
    r->tiles_total += fs.n_tiles;
    r->work_left += fs.tile_cost * fs.n_tiles;
}

// Order, id and admission of a validated request.
mc_status enqueue_request(mc_ctx* ctx, std::unique_ptr<Request> r, uint64_t* out_request_id)
{
    uint64_t parts = 0;
    for (const FnState& fs : r->st) parts += fs.n_tiles;
    if (parts > ctx->max_partials)
        return fail(ctx, MC_ERR_ADMISSION, "request needs %llu tile partials; the context holds %llu",
                    (unsigned long long)parts, (unsigned long long)ctx->max_partials);
    const size_t n = r->count();
    r->order.clear();
    for (size_t i = 0; i < n; ++i)
        if (r->st[i].next_tile < r->st[i].n_tiles) r->order.push_back((uint32_t)i);  // (a restored request: unfinished ones)
    Request* rq = r.get();
    std::stable_sort(rq->order.begin(), rq->order.end(),
                     [rq](uint32_t a, uint32_t b) { return rq->st[a].tile_cost > rq->st[b].tile_cost; });
    r->id = ctx->next_id++;
    *out_request_id = r->id;
    ctx->requests.emplace(rq->id, std::move(r));
    if (rq->fns_done == rq->count()) {  // a restored request whose results were all in
        ctx->completed.push_back(rq->id);
        return MC_OK;
    }
    if (!ctx->validate_only) {
        ctx->pending.push_back(rq);
        // The request is queued.  Admission is tried at once; if a HIP call of it
        // fails, the requests it was admitting stay queued as they were and the
        // next mc_run (which reports such failures) tries again.
        try {
            HIP_TRY(hipSetDevice(ctx->device));
            admit(ctx);
        } catch (const HipError&) {
        }
    }
    return MC_OK;
}

}  // namespace

mc_status mc_submit(mc_ctx* ctx, const mc_function* fns, size_t n, int32_t precision, uint64_t* out_request_id)
{
    if (!ctx) return fail(nullptr, MC_ERR_INVALID_ARG, "ctx is NULL");
    if (!fns || n == 0 || !out_request_id) return fail(ctx, MC_ERR_INVALID_ARG, "empty request or NULL argument");
    if (precision != MC_PREC_FP32_EVAL && precision != MC_PREC_FP64)
        return fail(ctx, MC_ERR_INVALID_ARG, "unknown precision %d", precision);
    if (n > ctx->max_functions)
        return fail(ctx, MC_ERR_ADMISSION, "request of %zu functions exceeds the %u function slots", n,
                    ctx->max_functions);
    std::unique_ptr<Request> r(new Request());
    r->precision = precision;
    r->fns.assign(fns, fns + n);
    r->n = n;
    r->st.resize(n);
    r->results.assign(n, mc_result{});
    for (size_t i = 0; i < n; ++i) {
        std::string why;
        mc_status st = validate_one(fns[i], ctx->n_user, &why);
        if (st != MC_OK) return fail(ctx, st, "function %zu: %s", i, why.c_str());
        const bool f64 = precision == MC_PREC_FP64 || (ctx->promote && fp32_hopeless(fns[i]));
        init_fn_state(ctx, r.get(), i, fns[i], f64);
    }
    // (records are packed at admission, into the pinned mirror of their slots)
    return enqueue_request(ctx, std::move(r), out_request_id);
}

mc_status mc_submit_grid(mc_ctx* ctx, const mc_function* base, const mc_grid_axis* axes, uint32_t n_axes,
                         int32_t precision, uint64_t* out_request_id)
{
    if (!ctx) return fail(nullptr, MC_ERR_INVALID_ARG, "ctx is NULL");
    if (!base || !axes || !out_request_id) return fail(ctx, MC_ERR_INVALID_ARG, "NULL argument");
    if (precision != MC_PREC_FP32_EVAL && precision != MC_PREC_FP64)
        return fail(ctx, MC_ERR_INVALID_ARG, "unknown precision %d", precision);
    if (n_axes < 1 || n_axes > MC_MAX_GRID_AXES)
        return fail(ctx, MC_ERR_INVALID_ARG, "n_axes %u outside 1..%d", n_axes, MC_MAX_GRID_AXES);
    uint64_t n = 1;
    for (uint32_t a = 0; a < n_axes; ++a) {
        if (axes[a].param >= (uint32_t)MC_N_PARAMS)
            return fail(ctx, MC_ERR_INVALID_ARG, "axis %u: param index %u above %d", a, axes[a].param, MC_N_PARAMS - 1);
        if (axes[a].count == 0) return fail(ctx, MC_ERR_INVALID_ARG, "axis %u: zero points", a);
        for (uint32_t b = 0; b < a; ++b)
            if (axes[b].param == axes[a].param)
                return fail(ctx, MC_ERR_INVALID_ARG, "axes %u and %u set the same parameter", b, a);
        n *= axes[a].count;
        if (n > ctx->max_functions)
            return fail(ctx, MC_ERR_ADMISSION, "grid of more than %u functions exceeds the context's function slots",
                        ctx->max_functions);
    }
    if (base->seed > UINT64_MAX - (n - 1))
        return fail(ctx, MC_ERR_INVALID_ARG, "seed range of the grid wraps 2^64");
    std::unique_ptr<Request> r(new Request());
    r->precision = precision;
    r->grid = true;
    r->n = n;
    r->spec.base = *base;
    for (uint32_t a = 0; a < n_axes; ++a) r->spec.axes[a] = axes[a];
    r->spec.n_axes = n_axes;
    r->spec.precision = precision;
    r->spec.n = n;
    // Validity without expanding the grid: every constraint involves one
    // parameter, so it suffices to check the grid's first point and, from
    // there, every point of each axis alone.
    {
        uint64_t stride = 1;
        std::string why;
        mc_function f;
        grid_function(r->spec.base, r->spec.axes, n_axes, 0, &f);
        mc_status st = validate_one(f, ctx->n_user, &why);
        if (st != MC_OK) return fail(ctx, st, "function 0: %s", why.c_str());
        for (uint32_t a = 0; a < n_axes; ++a) {
            for (uint32_t k = 1; k < axes[a].count; ++k) {
                grid_function(r->spec.base, r->spec.axes, n_axes, (uint64_t)k * stride, &f);
                st = validate_one(f, ctx->n_user, &why);
                if (st != MC_OK)
                    return fail(ctx, st, "function %llu: %s", (unsigned long long)((uint64_t)k * stride), why.c_str());
            }
            stride *= axes[a].count;
        }
    }
    // FP32 phase bound over the whole grid: each parameter at the end of its
    // axis with the larger magnitude (the bound grows with every |k_j|); a grid
    // that exceeds it anywhere is evaluated in FP64 throughout
    bool grid_f64 = precision == MC_PREC_FP64;
    if (!grid_f64 && ctx->promote) {
        mc_function fmax = r->spec.base;
        for (uint32_t a = 0; a < n_axes; ++a) {
            const double v0 = axes[a].start, v1 = axes[a].start + (double)(axes[a].count - 1) * axes[a].step;
            fmax.params[axes[a].param] = std::fabs(v1) > std::fabs(v0) ? v1 : v0;
        }
        grid_f64 = fp32_hopeless(fmax);
        if (grid_f64) r->spec.precision = MC_PREC_FP64;
    }
    // all functions share family, dimension and sample count: the base gives
    // everybody's schedule
    r->st.resize(n);
    r->results.assign(n, mc_result{});
    for (uint64_t i = 0; i < n; ++i) init_fn_state(ctx, r.get(), i, r->spec.base, grid_f64);
    return enqueue_request(ctx, std::move(r), out_request_id);
}

mc_status mc_run(mc_ctx* ctx, void* stream)
{
    if (!ctx) return fail(nullptr, MC_ERR_INVALID_ARG, "ctx is NULL");
    if (ctx->validate_only) return fail(ctx, MC_ERR_NO_DEVICE, "validate-only context has no device");
    bool no_slot = false;
    try {
        HIP_TRY(hipSetDevice(ctx->device));
        if (ctx->res.on) {
            res_step(ctx);
            return MC_OK;
        }
        hipStream_t s = (hipStream_t)stream;
        reap(ctx, 0);
        if (ctx->abort_requested) finish_abort(ctx);
        admit(ctx);
        launch(ctx, s, &no_slot);
    } catch (const HipError& e) {
        return fail_hip(ctx, e);
    }
    return no_slot ? MC_NOT_READY : MC_OK;
}

mc_status mc_poll(mc_ctx* ctx, uint64_t* completed, size_t cap, size_t* n)
{
    if (!ctx || !n || (cap > 0 && !completed)) return fail(ctx, MC_ERR_INVALID_ARG, "NULL argument");
    *n = 0;
    if (ctx->validate_only) return MC_OK;
    try {
        HIP_TRY(hipSetDevice(ctx->device));
        if (ctx->res.on) res_step(ctx);
        else reap(ctx, 0);
    } catch (const HipError& e) {
        return fail_hip(ctx, e);
    }
    while (*n < cap && !ctx->completed.empty()) {
        completed[(*n)++] = ctx->completed.front();
        ctx->completed.pop_front();
    }
    return MC_OK;
}

mc_status mc_pending(mc_ctx* ctx, uint64_t* requests, uint64_t* tiles)
{
    if (!ctx) return fail(nullptr, MC_ERR_INVALID_ARG, "ctx is NULL");
    uint64_t nr = 0, nt = 0;
    for (auto& kv : ctx->requests) {
        Request* r = kv.second.get();
        if (r->fns_done < r->count()) nr++;
        nt += r->tiles_total - r->tiles_launched;
    }
    if (requests) *requests = nr;
    if (tiles) *tiles = nt;
    return MC_OK;
}

mc_status mc_results(mc_ctx* ctx, uint64_t request_id, mc_result* out, size_t n, int blocking)
{
    if (!ctx) return fail(nullptr, MC_ERR_INVALID_ARG, "ctx is NULL");
    auto it = ctx->requests.find(request_id);
    if (it == ctx->requests.end())
        return fail(ctx, MC_ERR_UNKNOWN_REQUEST, "request %llu unknown or already taken", (unsigned long long)request_id);
    Request* r = it->second.get();
    if (!out || n != r->count())
        return fail(ctx, MC_ERR_INVALID_ARG, "request %llu has %zu functions, got n=%zu", (unsigned long long)request_id,
                    r->count(), n);
    if (ctx->validate_only) return fail(ctx, MC_ERR_NO_DEVICE, "validate-only context has no device");
    if (ctx->res.on) return res_results(ctx, it, out, n, blocking);
    try {
        HIP_TRY(hipSetDevice(ctx->device));
        reap(ctx, 0);
        while (r->fns_done < r->count()) {
            if (r->lost && !any_in_flight(ctx)) {
                // part of its work was lost with a failed launch; nothing in flight
                // refers to it any more, so it is released
                free_request_resources(ctx, r);
                ctx->requests.erase(it);
                return fail(ctx, MC_ERR_HIP, "request %llu cannot complete: its work was in a launch that failed",
                            (unsigned long long)request_id);
            }
            if (!blocking) return MC_NOT_READY;
            if (r->tiles_launched < r->tiles_total || has_work(r) || !r->admitted) {
                mc_status st = mc_run(ctx, nullptr);
                if (st == MC_NOT_READY) reap(ctx, 1);  // all slots busy: wait for the oldest launch
                else if (st != MC_OK) return st;
            } else if (any_in_flight(ctx)) {
                reap(ctx, 1);
            } else {
                // every tile was handed to a launch and every launch has been
                // reaped: the rest went to a launch that failed to enqueue.
                // Nothing in flight refers to the request, so it is released.
                free_request_resources(ctx, r);
                ctx->requests.erase(it);
                return fail(ctx, MC_ERR_HIP, "request %llu cannot complete: its work was in a launch that failed",
                            (unsigned long long)request_id);
            }
        }
    } catch (const HipError& e) {
        return fail_hip(ctx, e);
    }
    std::memcpy(out, r->results.data(), n * sizeof(mc_result));
    const bool aborted = r->aborted;
    ctx->requests.erase(it);
    return aborted ? MC_ERR_ABORTED : MC_OK;
}

mc_status mc_abort(mc_ctx* ctx)
{
    if (!ctx) return fail(nullptr, MC_ERR_INVALID_ARG, "ctx is NULL");
    if (ctx->validate_only) return MC_OK;
    if (ctx->res.on) {
        res_request_stop(ctx);
        ctx->abort_requested = true;
        ctx->abort_below = ctx->next_id;
        return MC_OK;
    }
    try {
        HIP_TRY(hipSetDevice(ctx->device));
        // The upload stream is non-blocking, so the word changes while kernels run.
        HIP_TRY(hipMemcpyAsync(ctx->d_abort_word, &ctx->h_words[1], sizeof(uint32_t), hipMemcpyHostToDevice,
                               ctx->upload_stream));
        HIP_TRY(hipStreamSynchronize(ctx->upload_stream));
        ctx->abort_requested = true;
        ctx->abort_below = ctx->next_id;
    } catch (const HipError& e) {
        return fail_hip(ctx, e);
    }
    return MC_OK;
}

mc_status mc_cancel(mc_ctx* ctx, uint64_t request_id)
{
    if (!ctx) return fail(nullptr, MC_ERR_INVALID_ARG, "ctx is NULL");
    auto it = ctx->requests.find(request_id);
    if (it == ctx->requests.end())
        return fail(ctx, MC_ERR_UNKNOWN_REQUEST, "request %llu unknown or already taken", (unsigned long long)request_id);
    Request* r = it->second.get();
    // a complete request keeps its results; a lost one reports its failure
    if (r->fns_done == r->count() || r->cancelled || r->lost) return MC_OK;
    auto drop_from = [r](std::deque<Request*>& q) {
        for (auto p = q.begin(); p != q.end(); ++p)
            if (*p == r) {
                q.erase(p);
                return;
            }
    };
    log_msg(2, "request %llu cancelled", (unsigned long long)request_id);
    if (!r->admitted) {
        drop_from(ctx->pending);
        complete_aborted(ctx, r);
        return MC_OK;
    }
    try {
        HIP_TRY(hipSetDevice(ctx->device));
        if (ctx->res.on) {
            ResidentState& R = ctx->res;
            R.tiles_waiting -= std::min<uint64_t>(R.tiles_waiting, r->tiles_total - r->tiles_launched);
            R.active_dirty = true;
        }
        r->cancelled = true;
        drop_work(r);
        drop_from(ctx->active);
        if (ctx->res.on) {
            res_cancel(ctx, r);
            if (!ctx->abort_requested) res_launch(ctx);  // (entries of other requests may wait)
        } else if (!in_flight_refers(ctx, r)) {
            complete_aborted(ctx, r);
        }
    } catch (const HipError& e) {
        return fail_hip(ctx, e);
    }
    return MC_OK;
}

// ---------------------------------------------------------------- checkpoint / resume
//
// Snapshot layout (native byte order):
//   SnapHeader | GridSpec (grids only) | mc_function[n] | SnapFn[n] | mc_result[n] | Partial[n_partials]
//   | uint32 n_sources, uint32 0 | per run-time family used: {uint32 id, uint32 0, uint64 length,
//     source text padded with zeros to a multiple of 8 bytes}
// partials: for each function in index order that has not finished, the
// partials of its tiles 0 .. next_tile.  A grid stays a grid (its records are
// packed on the device, which in FP32 need not match the host's packing bit
// for bit); its functions are listed too, and checked against the spec.  The
// sources of the run-time families the request uses let a restoring context
// find its own ids for them (it must have registered the same sources).
// Version 1 (no sources section) is read as well.

}  // extern "C"

namespace {

constexpr char kSnapMagic[8] = {'Z', 'M', 'C', 'S', 'N', 'A', 'P', '1'};

struct SnapHeader {
    char magic[8];
    uint32_t version;         // 2 (1: no sources section)
    uint32_t header_bytes;    // sizeof(SnapHeader)
    uint64_t total_bytes;
    uint64_t n;               // functions
    uint64_t n_partials;      // partials stored
    uint32_t seg_samples;     // tiling constants the partials were made with
    uint32_t block_waves;
    int32_t precision;
    uint32_t grid;            // 1: a parameter grid (GridSpec follows the header)
    uint64_t request_id;      // of the snapshotted request (for the reader's information)
};

struct SnapFn {
    uint32_t seg_log2;
    uint32_t n_tiles;
    uint32_t next_tile;       // tiles run; n_tiles when the result is in
    uint32_t f64;             // evaluated in FP64 (requested, or promoted)
};

static_assert(sizeof(SnapHeader) == 64 && sizeof(SnapFn) == 16, "snapshot layout");

uint64_t snapshot_bytes(uint64_t n, uint64_t n_partials, bool grid)
{
    return sizeof(SnapHeader) + (grid ? sizeof(GridSpec) : 0) +
           n * (sizeof(mc_function) + sizeof(SnapFn) + sizeof(mc_result)) + n_partials * sizeof(Partial);
}

// The run-time families request r uses, in increasing id order.
std::vector<uint32_t> user_families_of(const Request* r)
{
    std::vector<uint32_t> ids;
    auto add = [&ids](uint32_t fam) {
        if (fam >= kUserFamily0 && std::find(ids.begin(), ids.end(), fam) == ids.end()) ids.push_back(fam);
    };
    if (r->grid) add(r->spec.base.family);
    else
        for (const mc_function& f : r->fns) add(f.family);
    std::sort(ids.begin(), ids.end());
    return ids;
}

uint64_t sources_bytes(const mc_ctx* ctx, const std::vector<uint32_t>& ids)
{
    uint64_t b = 8;
    for (uint32_t id : ids) b += 16 + (ctx->user_src[id - kUserFamily0].size() + 7) / 8 * 8;
    return b;
}

}  // namespace

extern "C" {

mc_status mc_snapshot(mc_ctx* ctx, uint64_t request_id, void* buf, size_t cap, size_t* bytes)
{
    if (!ctx || !bytes) return fail(ctx, MC_ERR_INVALID_ARG, "NULL argument");
    auto it = ctx->requests.find(request_id);
    if (it == ctx->requests.end())
        return fail(ctx, MC_ERR_UNKNOWN_REQUEST, "request %llu unknown or already taken", (unsigned long long)request_id);
    Request* r = it->second.get();
    const uint64_t n = r->count();
    const std::vector<uint32_t> fams = user_families_of(r);
    std::vector<Partial> range;
    // each function's tiles run (resident: its open run's first tile still in
    // the ring)
    std::vector<uint32_t> ran(n), unread(n, UINT32_MAX);
    // a resident launch stopped for a snapshot written starts again on the way
    // out if entries wait (if that fails, the next step tries again); after a
    // size query it stays stopped until the next call that runs work, so the
    // size holds for the snapshot that follows
    struct Relaunch {
        mc_ctx* ctx = nullptr;
        ~Relaunch()
        {
            if (!ctx || ctx->abort_requested) return;
            try {
                res_launch(ctx);
            } catch (const HipError&) {
            }
        }
    } relaunch;
    try {
        if (!ctx->validate_only) {
            HIP_TRY(hipSetDevice(ctx->device));
            if (ctx->res.on) {
                // the resident launch stops and goes (every entry below the count
                // it last saw is run; from then on no kernel touches a partial),
                // results that came in are collected, and a run still open has
                // run its tiles up to its first chunk left unread in the ring
                // (a launch reads a prefix of the ring; a run's chunks are in it
                // in tile order)
                ResidentState& R = ctx->res;
                res_request_stop(ctx);
                res_wait_exit(ctx);
                res_reap(ctx);  // (may send results to FP64: progress is read after it)
                for (uint64_t e = R.acked; e < R.pushed && r->admitted; ++e) {
                    const Chunk& c = R.ring[e & (kRingEntries - 1)];
                    if (c.fn < r->slot_base || c.fn - r->slot_base >= n) continue;
                    const uint32_t i = c.fn - r->slot_base;
                    if (c.token == r->st[i].token) unread[i] = std::min(unread[i], c.first);
                }
            } else {
                reap(ctx, 2);  // every launch in flight: from here on no kernel touches its partials
            }
        }
        for (uint64_t i = 0; i < n; ++i) ran[i] = std::min(r->st[i].next_tile, unread[i]);
        if (r->lost || r->aborted)
            return fail(ctx, MC_ERR_INVALID_ARG, "request %llu was aborted or failed", (unsigned long long)request_id);
        uint64_t n_partials = 0;
        for (uint64_t i = 0; i < n; ++i) {
            const FnState& fs = r->st[i];
            if (fs.done) continue;
            ran[i] = std::min(ran[i], fs.n_tiles - 1);  // (a run whose result is not in has a tile left)
            n_partials += ran[i];
        }
        const uint64_t total = snapshot_bytes(n, n_partials, r->grid) + sources_bytes(ctx, fams);
        *bytes = (size_t)total;
        if (!buf) return MC_OK;
        if (cap < total)
            return fail(ctx, MC_ERR_INVALID_ARG, "snapshot needs %llu bytes, the buffer holds %zu",
                        (unsigned long long)total, cap);
        if (ctx->res.on && !ctx->validate_only) relaunch.ctx = ctx;
        if (n_partials > 0) {
            if (!r->admitted || r->partials_pending) {
                range = r->staged;  // a restored request whose saved partials are not on the device yet
            } else {
                // (on the stream that copied a restored request's saved partials up)
                hipStream_t st = ctx->res.on ? ctx->res.stream : ctx->upload_stream;
                range.resize(r->part_count);
                HIP_TRY(hipMemcpyAsync(range.data(), ctx->d_partials + r->part_base, r->part_count * sizeof(Partial),
                                       hipMemcpyDeviceToHost, st));
                HIP_TRY(hipStreamSynchronize(st));
            }
        }
        uint8_t* p = (uint8_t*)buf;
        SnapHeader h{};
        std::memcpy(h.magic, kSnapMagic, sizeof h.magic);
        h.version = 2;
        h.header_bytes = sizeof h;
        h.total_bytes = total;
        h.n = n;
        h.n_partials = n_partials;
        h.seg_samples = (uint32_t)kSegSamples;
        h.block_waves = (uint32_t)kBlockWaves;
        h.precision = r->precision;
        h.grid = r->grid ? 1u : 0u;
        h.request_id = r->id;
        std::memcpy(p, &h, sizeof h);
        p += sizeof h;
        if (r->grid) {
            std::memcpy(p, &r->spec, sizeof r->spec);
            p += sizeof r->spec;
        }
        for (uint64_t i = 0; i < n; ++i, p += sizeof(mc_function)) {
            const mc_function f = r->at(i);
            std::memcpy(p, &f, sizeof f);
        }
        for (uint64_t i = 0; i < n; ++i, p += sizeof(SnapFn)) {
            const FnState& fs = r->st[i];
            const SnapFn sf{fs.seg_log2, fs.n_tiles, fs.done ? fs.n_tiles : ran[i], fs.f64 ? 1u : 0u};
            std::memcpy(p, &sf, sizeof sf);
        }
        for (uint64_t i = 0; i < n; ++i, p += sizeof(mc_result)) {
            mc_result res{};
            if (r->st[i].done) res = r->results[i];
            std::memcpy(p, &res, sizeof res);
        }
        uint64_t off = 0;  // function i's first partial within the request's range
        for (uint64_t i = 0; i < n; ++i) {
            const FnState& fs = r->st[i];
            if (!fs.done && ran[i] > 0) {
                std::memcpy(p, range.data() + off, (size_t)ran[i] * sizeof(Partial));
                p += (size_t)ran[i] * sizeof(Partial);
            }
            off += fs.n_tiles;
        }
        const uint32_t head[2] = {(uint32_t)fams.size(), 0u};
        std::memcpy(p, head, sizeof head);
        p += sizeof head;
        for (uint32_t id : fams) {
            const std::string& text = ctx->user_src[id - kUserFamily0];
            const uint32_t idw[2] = {id, 0u};
            const uint64_t len = text.size();
            std::memcpy(p, idw, sizeof idw);
            std::memcpy(p + 8, &len, sizeof len);
            p += 16;
            const uint64_t padded = (len + 7) / 8 * 8;
            std::memset(p, 0, padded);
            std::memcpy(p, text.data(), len);
            p += padded;
        }
    } catch (const HipError& e) {
        return fail_hip(ctx, e);
    }
    log_msg(2, "request %llu snapshot: %llu bytes", (unsigned long long)request_id, (unsigned long long)*bytes);
    return MC_OK;
}

mc_status mc_restore(mc_ctx* ctx, const void* buf, size_t bytes, uint64_t* out_request_id)
{
    if (!ctx || !buf || !out_request_id) return fail(ctx, MC_ERR_INVALID_ARG, "NULL argument");
    SnapHeader h;
    if (bytes < sizeof h) return fail(ctx, MC_ERR_INVALID_ARG, "snapshot of %zu bytes is truncated", bytes);
    std::memcpy(&h, buf, sizeof h);
    if (std::memcmp(h.magic, kSnapMagic, sizeof h.magic) != 0 || (h.version != 1 && h.version != 2) ||
        h.header_bytes != sizeof h)
        return fail(ctx, MC_ERR_INVALID_ARG, "not a snapshot of this library version");
    if (h.seg_samples != (uint32_t)kSegSamples || h.block_waves != (uint32_t)kBlockWaves)
        return fail(ctx, MC_ERR_INVALID_ARG, "snapshot made with another tiling (%u samples per segment, %u waves)",
                    h.seg_samples, h.block_waves);
    if (h.n == 0 || h.n > ctx->max_functions)
        return fail(ctx, h.n == 0 ? MC_ERR_INVALID_ARG : MC_ERR_ADMISSION,
                    "snapshot of %llu functions; the context has %u function slots", (unsigned long long)h.n,
                    ctx->max_functions);
    const uint64_t body = h.grid > 1u || h.n > (1ull << 32) || h.n_partials > (1ull << 40)
                              ? UINT64_MAX
                              : snapshot_bytes(h.n, h.n_partials, h.grid != 0u);
    if (h.grid > 1u || h.n_partials > ctx->max_partials || h.total_bytes != bytes || body > bytes ||
        (h.version == 1 && body != bytes))
        return fail(ctx, MC_ERR_INVALID_ARG, "snapshot size %zu does not match its contents", bytes);
    // run-time families: the snapshot's ids mapped to this context's, by source text
    std::vector<std::pair<uint32_t, uint32_t>> fam_map;
    if (h.version == 2) {
        const uint8_t* q = (const uint8_t*)buf + body;
        const uint8_t* end = (const uint8_t*)buf + bytes;
        uint32_t head[2];
        if (end - q < 8) return fail(ctx, MC_ERR_INVALID_ARG, "snapshot size %zu does not match its contents", bytes);
        std::memcpy(head, q, sizeof head);
        q += 8;
        if (head[0] > (uint32_t)kMaxUserFamilies)
            return fail(ctx, MC_ERR_INVALID_ARG, "snapshot lists %u run-time families", head[0]);
        for (uint32_t k = 0; k < head[0]; ++k) {
            uint32_t idw[2];
            uint64_t len = 0;
            if (end - q < 16) return fail(ctx, MC_ERR_INVALID_ARG, "snapshot's family sources are truncated");
            std::memcpy(idw, q, sizeof idw);
            std::memcpy(&len, q + 8, sizeof len);
            q += 16;
            const uint64_t padded = (len + 7) / 8 * 8;
            if (len > (uint64_t)(end - q) || padded > (uint64_t)(end - q))
                return fail(ctx, MC_ERR_INVALID_ARG, "snapshot's family sources are truncated");
            const std::string text((const char*)q, (size_t)len);
            q += padded;
            size_t found = ctx->user_src.size();
            for (size_t u = 0; u < ctx->user_src.size(); ++u)
                if (ctx->user_src[u] == text) found = u;
            if (found == ctx->user_src.size())
                return fail(ctx, MC_ERR_UNSUPPORTED_FAMILY,
                            "the snapshot's run-time family %u is not registered on this context (register the "
                            "same source first)",
                            idw[0]);
            fam_map.emplace_back(idw[0], kUserFamily0 + (uint32_t)found);
        }
        if (q != end) return fail(ctx, MC_ERR_INVALID_ARG, "snapshot size %zu does not match its contents", bytes);
    }
    // (false: a run-time family the snapshot holds no source for)
    auto remap = [&fam_map](uint32_t* fam) {
        if (*fam < kUserFamily0) return true;
        for (const auto& m : fam_map)
            if (m.first == *fam) {
                *fam = m.second;
                return true;
            }
        return false;
    };
    if (h.precision != MC_PREC_FP32_EVAL && h.precision != MC_PREC_FP64)
        return fail(ctx, MC_ERR_INVALID_ARG, "snapshot precision %d", h.precision);
    const uint8_t* p = (const uint8_t*)buf + sizeof h;
    const uint64_t n = h.n;
    std::unique_ptr<Request> r(new Request());
    r->precision = h.precision;
    r->restored = true;
    r->n = n;
    if (h.grid) {
        std::memcpy(&r->spec, p, sizeof r->spec);
        p += sizeof r->spec;
        if (r->spec.n != n || r->spec.n_axes < 1 || r->spec.n_axes > (uint32_t)MC_MAX_GRID_AXES ||
            (r->spec.precision != MC_PREC_FP32_EVAL && r->spec.precision != MC_PREC_FP64) ||
            !remap(&r->spec.base.family))
            return fail(ctx, MC_ERR_INVALID_ARG, "snapshot's grid does not match its functions");
        r->grid = true;
    }
    r->fns.resize(n);
    std::memcpy(r->fns.data(), p, n * sizeof(mc_function));
    p += n * sizeof(mc_function);
    for (uint64_t i = 0; i < n; ++i)
        if (!remap(&r->fns[i].family))
            return fail(ctx, MC_ERR_INVALID_ARG, "function %llu: run-time family %u without its source",
                        (unsigned long long)i, r->fns[i].family);
    if (r->grid) {
        for (uint64_t i = 0; i < n; ++i) {
            mc_function g;
            grid_function(r->spec.base, r->spec.axes, r->spec.n_axes, i, &g);
            if (std::memcmp(&g, &r->fns[i], sizeof g) != 0)
                return fail(ctx, MC_ERR_INVALID_ARG, "snapshot's grid does not match function %llu",
                            (unsigned long long)i);
        }
    }
    std::vector<SnapFn> sf(n);
    std::memcpy(sf.data(), p, n * sizeof(SnapFn));
    p += n * sizeof(SnapFn);
    r->results.resize(n);
    std::memcpy(r->results.data(), p, n * sizeof(mc_result));
    p += n * sizeof(mc_result);
    const Partial* saved = (const Partial*)p;
    r->st.resize(n);
    uint64_t parts = 0, used = 0;
    for (uint64_t i = 0; i < n; ++i) {
        const mc_function& f = r->fns[i];
        std::string why;
        const mc_status st = validate_one(f, ctx->n_user, &why);
        if (st != MC_OK) return fail(ctx, st, "function %llu: %s", (unsigned long long)i, why.c_str());
        const uint32_t n_segments = (uint32_t)(((f.n_samples + 3) / 4 + kSegQuads - 1) / kSegQuads);
        const SnapFn& s = sf[i];
        if (s.seg_log2 > (uint32_t)kMaxSegLog2 || s.n_tiles != tiles_for(n_segments, s.seg_log2) ||
            s.next_tile > s.n_tiles || s.f64 > 1u || (h.precision == MC_PREC_FP64 && s.f64 == 0u))
            return fail(ctx, MC_ERR_INVALID_ARG, "function %llu: tiling or progress does not match the function",
                        (unsigned long long)i);
        FnState& fs = r->st[i];
        fs.seg_log2 = s.seg_log2;
        fs.n_tiles = s.n_tiles;
        fs.next_tile = s.next_tile;
        fs.f64 = s.f64 != 0u;
        fs.needs_upload = false;
        fs.token = 0;
        fs.rec = 0;
        fs.done = s.next_tile == s.n_tiles;
        fs.tile_cost = sample_cost(f.family, f.dim, fs.f64 ? MC_PREC_FP64 : MC_PREC_FP32_EVAL) *
                       (double)std::min<uint64_t>(f.n_samples, (uint64_t)kSegSamples * ((uint64_t)kBlockWaves << fs.seg_log2));
        if (s.next_tile == s.n_tiles) {
            const mc_result& res = r->results[i];
            if (res.status != MC_OK || res.n != f.n_samples ||
                res.precision != (fs.f64 ? (uint32_t)MC_PREC_FP64 : (uint32_t)MC_PREC_FP32_EVAL))
                return fail(ctx, MC_ERR_INVALID_ARG, "function %llu: its saved result does not match it",
                            (unsigned long long)i);
            r->fns_done++;
        } else {
            r->results[i] = mc_result{};
            r->tiles_total += fs.n_tiles;
            r->tiles_launched += fs.next_tile;
            r->work_left += fs.tile_cost * (double)(fs.n_tiles - fs.next_tile);
            used += fs.next_tile;
        }
        parts += fs.n_tiles;
    }
    if (used != h.n_partials)
        return fail(ctx, MC_ERR_INVALID_ARG, "snapshot holds %llu partials, its functions' progress needs %llu",
                    (unsigned long long)h.n_partials, (unsigned long long)used);
    if (parts > ctx->max_partials)
        return fail(ctx, MC_ERR_ADMISSION, "request needs %llu tile partials; the context holds %llu",
                    (unsigned long long)parts, (unsigned long long)ctx->max_partials);
    if (used > 0) {
        r->staged_counts.assign(n, 0u);
        for (uint64_t i = 0; i < n; ++i)
            if (r->st[i].next_tile < r->st[i].n_tiles) r->staged_counts[i] = r->st[i].next_tile;
        r->staged.assign(parts, Partial{0.0, 0.0});
        uint64_t off = 0, k = 0;
        for (uint64_t i = 0; i < n; ++i) {
            const FnState& fs = r->st[i];
            if (fs.next_tile < fs.n_tiles && fs.next_tile > 0) {
                std::memcpy(r->staged.data() + off, saved + k, (size_t)fs.next_tile * sizeof(Partial));
                k += fs.next_tile;
            }
            off += fs.n_tiles;
        }
    }
    if (r->grid) std::vector<mc_function>().swap(r->fns);  // (a grid's functions come from its spec)
    log_msg(2, "restoring a snapshot of request %llu: %llu functions, %llu finished, %llu partials",
            (unsigned long long)h.request_id, (unsigned long long)n, (unsigned long long)r->fns_done,
            (unsigned long long)used);
    return enqueue_request(ctx, std::move(r), out_request_id);
}

mc_status mc_integrate_plain_fp64(mc_ctx* ctx, const mc_function* fns, size_t n, mc_result* out, void* stream)
{
    if (!ctx) return fail(nullptr, MC_ERR_INVALID_ARG, "ctx is NULL");
    if (!fns || !out || n == 0) return fail(ctx, MC_ERR_INVALID_ARG, "empty request or NULL argument");
    if (ctx->validate_only) return fail(ctx, MC_ERR_NO_DEVICE, "validate-only context has no device");
    std::vector<DevFn> packed(n);
    uint64_t max_blocks = 1;
    for (size_t i = 0; i < n; ++i) {
        std::string why;
        mc_status st = validate_one(fns[i], 0, &why);  // built-in families only
        if (st != MC_OK) return fail(ctx, st, "function %zu: %s", i, why.c_str());
        pack_function(fns[i], MC_PREC_FP64, &packed[i]);
        const uint64_t blocks = (packed[i].n_quads + 255) / 256;
        if (blocks > 0x7FFFFFFFull) return fail(ctx, MC_ERR_INVALID_ARG, "function %zu: too many samples for one grid", i);
        max_blocks = std::max(max_blocks, blocks);
    }
    DevFn* d_fns = nullptr;
    Partial* d_parts = nullptr;
    DevResult* d_res = nullptr;
    mc_status status = MC_OK;
    try {
        HIP_TRY(hipSetDevice(ctx->device));
        hipStream_t s = (hipStream_t)stream;
        HIP_TRY(hipMalloc(&d_fns, n * sizeof(DevFn)));
        HIP_TRY(hipMalloc(&d_parts, max_blocks * sizeof(Partial)));
        HIP_TRY(hipMalloc(&d_res, n * sizeof(DevResult)));
        HIP_TRY(hipMemcpyAsync(d_fns, packed.data(), n * sizeof(DevFn), hipMemcpyHostToDevice, s));
        for (size_t i = 0; i < n; ++i) {
            const DevFn* f = d_fns + i;
            const uint32_t blocks = (uint32_t)((packed[i].n_quads + 255) / 256);
            void* a1[] = {&f, &d_parts};
            HIP_TRY(hipLaunchKernel(plain_kernel_ptr(), dim3(blocks), dim3(256), a1, 0, s));
            DevResult* r = d_res + i;
            void* a2[] = {&f, &d_parts, (void*)&blocks, &r};
            HIP_TRY(hipLaunchKernel(plain_reduce_kernel_ptr(), dim3(1), dim3(256), a2, 0, s));
        }
        HIP_TRY(hipMemcpyAsync(out, d_res, n * sizeof(DevResult), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    } catch (const HipError& e) {
        status = fail_hip(ctx, e);
    }
    if (d_fns) quiet(hipFree(d_fns));
    if (d_parts) quiet(hipFree(d_parts));
    if (d_res) quiet(hipFree(d_res));
    return status;
}

mc_status mc_integrate_plain_fp64_noalloc(mc_ctx* ctx, const mc_function* fns, size_t n, mc_result* out,
                                          void* stream)
{
    if (!ctx) return fail(nullptr, MC_ERR_INVALID_ARG, "ctx is NULL");
    if (!fns || !out || n == 0) return fail(ctx, MC_ERR_INVALID_ARG, "empty request or NULL argument");
    if (ctx->validate_only) return fail(ctx, MC_ERR_NO_DEVICE, "validate-only context has no device");
    if (n > kNoAllocMaxFunctions)
        return fail(ctx, MC_ERR_INVALID_ARG, "%zu functions exceed the no-allocation limit of %u", n,
                    kNoAllocMaxFunctions);
    uint64_t max_blocks = 1;
    for (size_t i = 0; i < n; ++i) {
        std::string why;
        const mc_status st = validate_one(fns[i], 0, &why);  // built-in families only
        if (st != MC_OK) return fail(ctx, st, "function %zu: %s", i, why.c_str());
        const uint64_t blocks = ((fns[i].n_samples + 3) / 4 + 255) / 256;
        if (blocks > kNoAllocMaxBlocks)
            return fail(ctx, MC_ERR_INVALID_ARG, "function %zu: %llu samples exceed the no-allocation limit of 2^30", i,
                        (unsigned long long)fns[i].n_samples);
        max_blocks = std::max(max_blocks, blocks);
    }
    // working set in `scratch`: [caller's table | records | results | block partials]
    const uint64_t rec_off = align256((uint64_t)n * sizeof(mc_function));
    const uint64_t res_off = rec_off + (uint64_t)n * sizeof(DevFn);
    const uint64_t part_off = res_off + align256((uint64_t)n * sizeof(DevResult));
    if (part_off + max_blocks * sizeof(Partial) > kScratchBytes)
        return fail(ctx, MC_ERR_INVALID_ARG, "no-allocation working set exceeds %llu bytes",
                    (unsigned long long)kScratchBytes);
    try {
        HIP_TRY(hipSetDevice(ctx->device));
        hipStream_t s = (hipStream_t)stream;
        uint8_t* const base = ctx->scratch;
        mc_function* d_table = (mc_function*)base;
        DevFn* d_fns = (DevFn*)(base + rec_off);
        DevResult* d_res = (DevResult*)(base + res_off);
        Partial* d_parts = (Partial*)(base + part_off);
        HIP_TRY(hipMemcpyAsync(d_table, fns, n * sizeof(mc_function), hipMemcpyHostToDevice, s));
        uint32_t n32 = (uint32_t)n;
        int32_t prec = MC_PREC_FP64;
        void* pa[] = {&d_table, &n32, &prec, &d_fns};
        HIP_TRY(hipLaunchKernel(pack_table_kernel_ptr(), dim3((n32 + 255) / 256), dim3(256), pa, 0, s));
        // every block of the plain kernel writes its partial and the reduction
        // reads exactly those: nothing in `scratch` has to start at zero
        for (size_t i = 0; i < n; ++i) {
            const DevFn* f = d_fns + i;
            const uint32_t blocks = (uint32_t)(((fns[i].n_samples + 3) / 4 + 255) / 256);
            void* a1[] = {&f, &d_parts};
            HIP_TRY(hipLaunchKernel(plain_kernel_ptr(), dim3(blocks), dim3(256), a1, 0, s));
            DevResult* r = d_res + i;
            void* a2[] = {&f, &d_parts, (void*)&blocks, &r};
            HIP_TRY(hipLaunchKernel(plain_reduce_kernel_ptr(), dim3(1), dim3(256), a2, 0, s));
        }
        HIP_TRY(hipMemcpyAsync(out, d_res, n * sizeof(DevResult), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    } catch (const HipError& e) {
        return fail_hip(ctx, e);
    }
    return MC_OK;
}

mc_status mc_sample_points(mc_ctx* ctx, const mc_function* f, uint64_t first, uint64_t count, double* out,
                           void* stream)
{
    if (!ctx) return fail(nullptr, MC_ERR_INVALID_ARG, "ctx is NULL");
    if (!f || !out || count == 0) return fail(ctx, MC_ERR_INVALID_ARG, "NULL argument or empty range");
    if (ctx->validate_only) return fail(ctx, MC_ERR_NO_DEVICE, "validate-only context has no device");
    std::string why;
    const mc_status st = validate_one(*f, ctx->n_user, &why);
    if (st != MC_OK) return fail(ctx, st, "function: %s", why.c_str());
    if (count > (1ull << 26)) return fail(ctx, MC_ERR_INVALID_ARG, "count %llu above 2^26", (unsigned long long)count);
    if (first >= f->n_samples || count > f->n_samples - first)
        return fail(ctx, MC_ERR_INVALID_ARG, "samples [%llu, %llu) outside 0..%llu", (unsigned long long)first,
                    (unsigned long long)(first + count), (unsigned long long)f->n_samples);
    DevFn packed;
    pack_function(*f, MC_PREC_FP64, &packed);
    DevFn* d_fn = nullptr;
    double* d_out = nullptr;
    const size_t out_bytes = (size_t)count * f->dim * sizeof(double);
    mc_status status = MC_OK;
    try {
        HIP_TRY(hipSetDevice(ctx->device));
        hipStream_t s = (hipStream_t)stream;
        HIP_TRY(hipMalloc(&d_fn, sizeof(DevFn)));
        HIP_TRY(hipMalloc(&d_out, out_bytes));
        HIP_TRY(hipMemcpyAsync(d_fn, &packed, sizeof(DevFn), hipMemcpyHostToDevice, s));
        void* args[] = {&d_fn, &first, &count, &d_out};
        HIP_TRY(hipLaunchKernel(sample_points_kernel_ptr(), dim3((unsigned)((count + 255) / 256)), dim3(256), args, 0, s));
        HIP_TRY(hipMemcpyAsync(out, d_out, out_bytes, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    } catch (const HipError& e) {
        status = fail_hip(ctx, e);
    }
    if (d_fn) quiet(hipFree(d_fn));
    if (d_out) quiet(hipFree(d_out));
    return status;
}

mc_status mc_get_tuning(mc_ctx* ctx, uint32_t* blocks_per_cu, uint8_t* seg_log2)
{
    if (!ctx) return fail(nullptr, MC_ERR_INVALID_ARG, "ctx is NULL");
    if (blocks_per_cu) *blocks_per_cu = ctx->blocks_per_cu32;
    if (seg_log2)
        for (int p = 0; p < 2; ++p)
            for (int f = 0; f < 4; ++f)
                for (int d = 0; d < kMaxDim; ++d) seg_log2[(p * 4 + f) * kMaxDim + d] = ctx->seg_log2[p][f][d];
    return MC_OK;
}

mc_status mc_set_tuning(mc_ctx* ctx, uint32_t blocks_per_cu, const uint8_t* seg_log2)
{
    if (!ctx) return fail(nullptr, MC_ERR_INVALID_ARG, "ctx is NULL");
    if (blocks_per_cu > 32) return fail(ctx, MC_ERR_INVALID_ARG, "blocks_per_cu %u > 32", blocks_per_cu);
    if (seg_log2) {
        for (int i = 0; i < 2 * 4 * kMaxDim; ++i)
            if (seg_log2[i] > kMaxSegLog2) return fail(ctx, MC_ERR_INVALID_ARG, "seg_log2 entry %d > %d", i, kMaxSegLog2);
        for (int p = 0; p < 2; ++p)
            for (int f = 0; f < 4; ++f)
                for (int d = 0; d < kMaxDim; ++d) ctx->seg_log2[p][f][d] = seg_log2[(p * 4 + f) * kMaxDim + d];
    }
    if (blocks_per_cu) {
        ctx->blocks_per_cu32 = blocks_per_cu;
        // graphs bake the grid size in: recapture lazily
        for (auto& s : ctx->slots) {
            if (s.in_flight && s.ev) quiet(hipEventSynchronize(s.ev->done));
            if (s.graph) {
                quiet(hipGraphExecDestroy(s.graph));
                s.graph = nullptr;
            }
        }
        try {
            reap(ctx, 2);
        } catch (const HipError& e) {
            return fail_hip(ctx, e);
        }
    }
    return MC_OK;
}


// Synthetic function of a given class for tuning trials (unit box, moderate parameters).
static mc_function tune_function(uint32_t family, uint32_t dim, uint64_t n_samples, uint64_t seed, bool high_degree)
{
    mc_function f;
    std::memset(&f, 0, sizeof f);
    f.family = family;
    f.dim = dim;
    f.n_samples = n_samples;
    f.seed = seed;
    for (uint32_t j = 0; j < dim; ++j) {
        f.lo[j] = 0.0;
        f.hi[j] = 1.0;
    }
    f.params[0] = 1.0;
    f.params[1] = family == MC_FAMILY_GAUSSIAN ? 0.5 : 0.5;
    for (uint32_t j = 0; j < dim; ++j) {
        f.params[MC_PARAM_V0 + j] = family == MC_FAMILY_POLY_PRODUCT ? 0.5 : 3.0;
        f.params[MC_PARAM_W0 + j] = family == MC_FAMILY_POLY_PRODUCT ? (high_degree ? 6.0 : 3.0) : 0.0;
    }
    return f;
}

// Time one batch through the normal path; returns the persistent-kernel milliseconds.
static double time_batch(mc_ctx* ctx, const std::vector<mc_function>& fns, int32_t precision, hipStream_t stream)
{
    uint64_t id = 0;
    if (mc_submit(ctx, fns.data(), fns.size(), precision, &id) != MC_OK) return -1.0;
    double total = 0.0;
    auto it = ctx->requests.find(id);
    Request* r = it->second.get();
    for (int guard = 0; guard < 64 && r->fns_done < r->count(); ++guard) {
        if (mc_run(ctx, stream) != MC_OK) return -1.0;
        reap(ctx, 2);
        collect_all_timing(ctx);
        total += ctx->last_main_ms;
    }
    std::vector<mc_result> out(fns.size());
    if (mc_results(ctx, id, out.data(), out.size(), 1) != MC_OK) return -1.0;
    return total;
}

}  // extern "C"

namespace {

mc_status autotune_run(mc_ctx* ctx, int32_t precision, void* stream, double budget_seconds);

// Tuning cache (MC_TUNE_CACHE names a text file): one line per device kind,
// compute-unit count, library version and precision,
//   zmc-tune 1 <arch> <CUs> <version> <precision> <blocks per CU> <48 seg_log2 values>
// where the values are the [2][4][12] table of mc_get_tuning.  Results never
// depend on the tuning, so a stale or foreign line can only cost speed.
std::string tune_key(const mc_ctx* ctx, int precision)
{
    char buf[256];
    snprintf(buf, sizeof buf, "zmc-tune 1 %s %d %s %d", ctx->device_name.c_str(), ctx->num_cus, mc_version(), precision);
    for (char& c : buf)
        if (c == '\n') c = ' ';
    return buf;
}

bool load_tuning(mc_ctx* ctx, const char* path, int precision)
{
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    const std::string key = tune_key(ctx, precision);
    // later lines override earlier ones (a re-tuned context appends)
    bool found = false;
    uint32_t blocks = 0;
    uint8_t seg[2 * 4 * kMaxDim] = {};
    char line[1024];
    while (std::fgets(line, sizeof line, f)) {
        std::string l(line);
        if (l.compare(0, key.size(), key) != 0 || l.size() <= key.size() || l[key.size()] != ' ') continue;
        const char* q = l.c_str() + key.size();
        char* end = nullptr;
        const unsigned long b = std::strtoul(q, &end, 10);
        if (end == q || b < 1 || b > 32) continue;
        uint8_t v[2 * 4 * kMaxDim];
        bool ok = true;
        for (int i = 0; i < 2 * 4 * kMaxDim && ok; ++i) {
            q = end;
            const unsigned long x = std::strtoul(q, &end, 10);
            ok = end != q && x <= (unsigned long)kMaxSegLog2;
            v[i] = (uint8_t)x;
        }
        if (!ok) continue;
        found = true;
        blocks = (uint32_t)b;
        std::memcpy(seg, v, sizeof seg);
    }
    std::fclose(f);
    if (!found) return false;
    // the cached line holds the tuned precision's rows; keep the other precision's
    uint8_t cur[2 * 4 * kMaxDim];
    mc_get_tuning(ctx, nullptr, cur);
    const int p = precision == MC_PREC_FP64 ? 1 : 0;
    std::memcpy(cur + p * 4 * kMaxDim, seg + p * 4 * kMaxDim, 4 * kMaxDim);
    return mc_set_tuning(ctx, precision == MC_PREC_FP32_EVAL ? blocks : 0, cur) == MC_OK;
}

void store_tuning(mc_ctx* ctx, const char* path, int precision)
{
    uint32_t blocks = 0;
    uint8_t seg[2 * 4 * kMaxDim];
    mc_get_tuning(ctx, &blocks, seg);
    std::string text = tune_key(ctx, precision) + " " + std::to_string(blocks);
    for (int i = 0; i < 2 * 4 * kMaxDim; ++i) text += " " + std::to_string((unsigned)seg[i]);
    text += "\n";
    FILE* f = std::fopen(path, "a");
    if (!f) return;  // the cache is an optimisation: a file that cannot be written is ignored
    std::fputs(text.c_str(), f);
    std::fclose(f);
}

}  // namespace

extern "C" mc_status mc_autotune(mc_ctx* ctx, int32_t precision, void* stream, double budget_seconds)
{
    if (!ctx) return fail(nullptr, MC_ERR_INVALID_ARG, "ctx is NULL");
    if (ctx->validate_only) return fail(ctx, MC_ERR_NO_DEVICE, "validate-only context has no device");
    if (precision != MC_PREC_FP32_EVAL && precision != MC_PREC_FP64)
        return fail(ctx, MC_ERR_INVALID_ARG, "unknown precision %d", precision);
    const char* cache = std::getenv("MC_TUNE_CACHE");
    if (cache && *cache && load_tuning(ctx, cache, precision)) {
        log_msg(2, "tuning (precision %d) from %s: %u workgroups per CU", (int)precision, cache,
                precision == MC_PREC_FP64 ? ctx->blocks_per_cu64 : ctx->blocks_per_cu32);
        return MC_OK;
    }
    if (ctx->res.on)
        return fail(ctx, MC_ERR_INVALID_ARG,
                    "a resident context does not time launches: tune a launch context (with MC_TUNE_CACHE) first");
    const mc_status st = autotune_run(ctx, precision, stream, budget_seconds);
    if (st == MC_OK && cache && *cache) store_tuning(ctx, cache, precision);
    if (st == MC_OK)
        log_msg(2, "tuning (precision %d): %u workgroups per CU", (int)precision,
                precision == MC_PREC_FP64 ? ctx->blocks_per_cu64 : ctx->blocks_per_cu32);
    return st;
}

namespace {

mc_status autotune_run(mc_ctx* ctx, int32_t precision, void* stream, double budget_seconds)
{
    const auto t0 = std::chrono::steady_clock::now();
    auto elapsed = [&] { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); };
    hipStream_t s = (hipStream_t)stream;
    const int p = precision == MC_PREC_FP64 ? 1 : 0;
    // Trials fill the chip many times over (a few ms of kernel time each), so
    // the tail of a launch does not decide; each is the best of `reps` runs.
    const uint32_t n_fns = (uint32_t)std::max(64, ctx->num_cus) * 8u;
    const int reps = 3;
    auto best_of = [&](const std::vector<mc_function>& fns) {
        double t = 1e30;
        for (int r = 0; r < reps; ++r) {
            const double x = time_batch(ctx, fns, precision, s);
            if (x > 0 && x < t) t = x;
        }
        return t;
    };
    // 1) workgroups per CU (FP32 kernel), on a 4-D harmonic batch of 2^20 samples per function
    if (p == 0) {
        int occ = 0;
        quiet(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, batched_kernel_ptr(false), kBlockThreads, 0));
        uint32_t best_b = ctx->blocks_per_cu32;
        double best_t = 1e30;
        std::vector<mc_function> fns;
        for (uint32_t i = 0; i < n_fns; ++i) fns.push_back(tune_function(MC_FAMILY_HARMONIC, 4, 1u << 20, i, false));
        for (int b = std::max(1, occ); b >= 1 && elapsed() < budget_seconds * 0.3; --b) {
            if (mc_set_tuning(ctx, (uint32_t)b, nullptr) != MC_OK) break;
            time_batch(ctx, fns, precision, s);  // warm-up (graph capture)
            const double t = best_of(fns);
            if (t < best_t * 0.99) {  // fewer workgroups must win by more than noise
                best_t = t;
                best_b = (uint32_t)b;
            }
        }
        mc_set_tuning(ctx, best_b, nullptr);
    }
    // 2) segments per wave per tile, per (family, dim)
    const uint32_t dims[] = {1, 2, 3, 4, 6, 8, 12};
    const int nfam = kNumFamilies;
    for (int fam = 0; fam < nfam && elapsed() < budget_seconds; ++fam) {
        for (uint32_t di = 0; di < sizeof(dims) / sizeof(dims[0]) && elapsed() < budget_seconds; ++di) {
            const uint32_t dim = dims[di];
            std::vector<mc_function> fns;
            const uint32_t family = (uint32_t)fam;
            const uint64_t n = (uint64_t)(4u << 20) / dim;
            for (uint32_t i = 0; i < n_fns / 4; ++i) fns.push_back(tune_function(family, dim, n, i, false));
            int best_l = 0;
            double best_t = 1e30;
            for (int l = 0; l <= 3; ++l) {
                ctx->seg_log2[p][fam][dim - 1] = (uint8_t)l;
                const double t = best_of(fns);
                if (t < best_t * 0.98) {
                    best_t = t;
                    best_l = l;
                }
            }
            // apply to this dim and the untested dims up to the next tested one
            const uint32_t next = di + 1 < sizeof(dims) / sizeof(dims[0]) ? dims[di + 1] : kMaxDim + 1;
            for (uint32_t d = dim; d < next; ++d) ctx->seg_log2[p][fam][d - 1] = (uint8_t)best_l;
        }
    }
    return MC_OK;
}

}  // namespace

extern "C" {

mc_status mc_last_run_timing(mc_ctx* ctx, double* main_ms, double* finalize_ms)
{
    if (!ctx) return fail(nullptr, MC_ERR_INVALID_ARG, "ctx is NULL");
    if (!ctx->validate_only) {
        quiet(hipSetDevice(ctx->device));
        collect_all_timing(ctx);
    }
    if (!ctx->have_timing) return fail(ctx, MC_NOT_READY, "no completed run yet");
    if (main_ms) *main_ms = ctx->last_main_ms;
    if (finalize_ms) *finalize_ms = ctx->last_fin_ms;
    return MC_OK;
}

mc_status mc_get_stats(mc_ctx* ctx, mc_stats* out)
{
    if (!ctx || !out) return fail(ctx, MC_ERR_INVALID_ARG, "NULL argument");
    if (!ctx->validate_only) {
        // timings of completed launches whose events the runtime had not yet released
        quiet(hipSetDevice(ctx->device));
        collect_all_timing(ctx);
    }
    *out = ctx->stats;
    return MC_OK;
}

}  // extern "C"

namespace {

// Source of the run-time kernels of one family: the caller's integrand wrapped
// in the evaluator interface, and the FP32 and FP64 persistent kernels that
// fetch only this family's part of a launch's tile list.
std::string user_family_source(const char* user_source, uint32_t family, uint32_t kidx32)
{
    std::string src;
    src += "#include \"zmc_device_code.hpp\"\n";
    src += "namespace zmc_user {\n#line 1 \"integrand\"\n";
    src += user_source;
    src += "\n}  // namespace zmc_user\n";
    src += "struct ZmcUserFn {\n"
           "    template <class T>\n"
           "    static __device__ __forceinline__ T f(const T* x, const T* p, uint32_t d)\n"
           "    { return zmc_user::mc_user_integrand<T>(x, p, d); }\n"
           "};\n";
    char buf[512];
    snprintf(buf, sizeof buf,
             "extern \"C\" __global__ __launch_bounds__(%d) void zmc_user_fp32(const zmc::LaunchDesc* __restrict__ Ld)\n"
             "{ zmc::batched_body<zmc::UserDispatch<ZmcUserFn, %uu, false>>(Ld, %uu); }\n"
             "extern \"C\" __global__ __launch_bounds__(%d) void zmc_user_fp64(const zmc::LaunchDesc* __restrict__ Ld)\n"
             "{ zmc::batched_body<zmc::UserDispatch<ZmcUserFn, %uu, true>>(Ld, %uu); }\n",
             kBlockThreads, family, kidx32, kBlockThreads, family, kidx32 + 1);
    src += buf;
    return src;
}

// Source of the resident kernel of a context with run-time families: every
// family registered so far in its own namespace, and a dispatch that tries the
// built-in families, then each of them.
std::string resident_user_source(const std::vector<std::string>& sources)
{
    std::string src = "#include \"zmc_device_code.hpp\"\n";
    char buf[512];
    for (size_t k = 0; k < sources.size(); ++k) {
        snprintf(buf, sizeof buf, "namespace zmc_user_%zu {\n#line 1 \"integrand %zu\"\n", k, k);
        src += buf;
        src += sources[k];
        snprintf(buf, sizeof buf,
                 "\n}  // namespace zmc_user_%zu\n"
                 "struct ZmcUserFn%zu {\n"
                 "    template <class T>\n"
                 "    static __device__ __forceinline__ T f(const T* x, const T* p, uint32_t d)\n"
                 "    { return zmc_user_%zu::mc_user_integrand<T>(x, p, d); }\n"
                 "};\n",
                 k, k, k);
        src += buf;
    }
    src += "template <bool F64>\n"
           "struct ZmcResidentDispatch {\n"
           "    __device__ static __forceinline__ bool run(zmc::CDevFn* fn, uint32_t fam, uint32_t seg0, uint32_t seg_log2,\n"
           "                                               uint32_t wave, uint32_t lane, zmc::Partial* s_seg)\n"
           "    {\n"
           "        if (zmc::BuiltinDispatch<F64>::run(fn, fam, seg0, seg_log2, wave, lane, s_seg)) return true;\n";
    for (size_t k = 0; k < sources.size(); ++k) {
        snprintf(buf, sizeof buf,
                 "        if (zmc::UserDispatch<ZmcUserFn%zu, %uu, F64>::run(fn, fam, seg0, seg_log2, wave, lane, s_seg))"
                 " return true;\n",
                 k, kUserFamily0 + (uint32_t)k);
        src += buf;
    }
    src += "        return false;\n"
           "    }\n"
           "};\n";
    snprintf(buf, sizeof buf,
             "extern \"C\" __global__ __launch_bounds__(%d) void zmc_resident_user(const zmc::ResidentDesc* __restrict__ R,"
             " uint32_t epoch)\n"
             "{ zmc::resident_body<ZmcResidentDispatch<false>, ZmcResidentDispatch<true>>(R, epoch); }\n",
             kBlockThreads);
    src += buf;
    return src;
}

// Code objects compiled in this process, by source text (the library's headers
// and compile options are fixed for a build): contexts that register the same
// families compile them once.  Failed compiles are not kept.
std::mutex g_rtc_mu;
std::map<std::string, std::vector<char>> g_rtc_cache;

bool compile_uncached(const std::string& src, std::vector<char>* code, std::string* log);

// Compile with hipRTC for gfx950; returns the code object or sets *log.
bool compile_user_family(const std::string& src, std::vector<char>* code, std::string* log)
{
    {
        std::lock_guard<std::mutex> lock(g_rtc_mu);
        auto it = g_rtc_cache.find(src);
        if (it != g_rtc_cache.end()) {
            *code = it->second;
            log_msg(2, "run-time family: code object reused (%zu bytes)", code->size());
            return true;
        }
    }
    if (!compile_uncached(src, code, log)) return false;
    std::lock_guard<std::mutex> lock(g_rtc_mu);
    g_rtc_cache.emplace(src, *code);
    return true;
}

bool compile_uncached(const std::string& src, std::vector<char>* code, std::string* log)
{
    hiprtcProgram prog = nullptr;
    const char* hdr_src[] = {kRtcHeaderDevice, kRtcHeaderCode};
    const char* hdr_name[] = {"zmc_device.hpp", "zmc_device_code.hpp"};
    if (hiprtcCreateProgram(&prog, src.c_str(), "zmc_user_family.hip", 2, hdr_src, hdr_name) != HIPRTC_SUCCESS) {
        *log = "hiprtcCreateProgram failed";
        return false;
    }
    // the same code generation as the built-in kernels
    const char* opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off", "-Xclang",
                          "-target-feature", "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult rc = hiprtcCompileProgram(prog, (int)(sizeof opts / sizeof opts[0]), opts);
    size_t log_size = 0;
    hiprtcGetProgramLogSize(prog, &log_size);
    std::string text(log_size, '\0');
    if (log_size) hiprtcGetProgramLog(prog, &text[0]);
    while (!text.empty() && text.back() == '\0') text.pop_back();
    bool ok = rc == HIPRTC_SUCCESS;
    if (ok) {
        size_t n = 0;
        ok = hiprtcGetCodeSize(prog, &n) == HIPRTC_SUCCESS && n > 0;
        if (ok) {
            code->resize(n);
            ok = hiprtcGetCode(prog, code->data()) == HIPRTC_SUCCESS;
        }
    }
    if (!ok) *log = std::string(hiprtcGetErrorString(rc)) + (text.empty() ? "" : ":\n" + text);
    hiprtcDestroyProgram(&prog);
    return ok;
}

// mc_register_family on a resident context: the resident kernel is compiled
// again with every family registered so far and this one; the running launch
// (of the previous kernel) is stopped and has gone before the new kernel
// replaces it, and launches again at once if entries wait.
mc_status register_resident_family(mc_ctx* ctx, const char* source, uint32_t* family_out)
{
    ResidentState& R = ctx->res;
    std::vector<std::string> all = ctx->user_src;
    all.push_back(source);
    std::vector<char> code;
    std::string log;
    if (!compile_user_family(resident_user_source(all), &code, &log)) {
        ctx->err = "run-time family did not compile: " + log;
        g_thread_error = ctx->err;
        return MC_ERR_COMPILE;
    }
    if (!ctx->validate_only) {
        hipModule_t module = nullptr;
        try {
            hipFunction_t kernel = nullptr;
            int occ = 0;
            HIP_TRY(hipSetDevice(ctx->device));
            HIP_TRY(hipModuleLoadData(&module, code.data()));
            HIP_TRY(hipModuleGetFunction(&kernel, module, "zmc_resident_user"));
            HIP_TRY(hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, kBlockThreads, 0));
            res_request_stop(ctx);
            res_wait_exit(ctx);
            HIP_TRY(hipStreamSynchronize(R.stream));
            if (R.user_module) quiet(hipModuleUnload(R.user_module));
            R.user_module = module;
            R.user_kernel = kernel;
            module = nullptr;
            const mc_config& cfg = ctx->cfg;
            R.grid = (uint32_t)ctx->num_cus * (cfg.blocks_per_cu ? cfg.blocks_per_cu : (uint32_t)std::max(1, occ));
            if (!cfg.max_tiles_per_run) R.backlog = 2ull * R.grid;  // (as at creation)
            log_msg(2, "resident kernel compiled with %zu run-time families: %u workgroups", all.size(), R.grid);
            if (!ctx->abort_requested) res_launch(ctx);  // (entries may wait)
        } catch (const HipError& e) {
            if (module) quiet(hipModuleUnload(module));
            return fail_hip(ctx, e);
        }
    }
    ctx->user_src.push_back(source);
    *family_out = kUserFamily0 + ctx->n_user;
    ctx->n_user++;
    return MC_OK;
}

}  // namespace

extern "C" {

mc_status mc_register_family(mc_ctx* ctx, const char* source, uint32_t* family_out)
{
    if (!ctx) return fail(nullptr, MC_ERR_INVALID_ARG, "ctx is NULL");
    if (!source || !family_out) return fail(ctx, MC_ERR_INVALID_ARG, "NULL argument");
    if (ctx->n_user >= (uint32_t)kMaxUserFamilies)
        return fail(ctx, MC_ERR_INVALID_ARG, "at most %d run-time families per context", kMaxUserFamilies);
    const uint32_t u = ctx->n_user;
    const uint32_t family = kUserFamily0 + u;
    if (ctx->res.on) return register_resident_family(ctx, source, family_out);
    const std::string src = user_family_source(source, family, 2 + 2 * u);
    std::vector<char> code;
    std::string log;
    if (!compile_user_family(src, &code, &log)) {
        ctx->err = "run-time family did not compile: " + log;
        g_thread_error = ctx->err;
        return MC_ERR_COMPILE;
    }
    if (!ctx->validate_only) {
        mc_ctx::UserFamily uf;
        try {
            HIP_TRY(hipSetDevice(ctx->device));
            HIP_TRY(hipModuleLoadData(&uf.module, code.data()));
            HIP_TRY(hipModuleGetFunction(&uf.kernel[0], uf.module, "zmc_user_fp32"));
            HIP_TRY(hipModuleGetFunction(&uf.kernel[1], uf.module, "zmc_user_fp64"));
            for (int p = 0; p < 2; ++p) {
                int occ = 0;
                HIP_TRY(hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&occ, uf.kernel[p], kBlockThreads, 0));
                uf.blocks_per_cu[p] = (uint32_t)std::max(1, occ);
            }
        } catch (const HipError& e) {
            if (uf.module) quiet(hipModuleUnload(uf.module));
            return fail_hip(ctx, e);
        }
        ctx->user[u] = uf;
    }
    ctx->user_src.push_back(source);
    ctx->n_user = u + 1;
    *family_out = family;
    return MC_OK;
}

const char* mc_last_error(mc_ctx* ctx)
{
    if (ctx) return ctx->err.c_str();
    return g_thread_error.c_str();
}

uint32_t mc_segment_samples(void) { return (uint32_t)kSegSamples; }

const char* mc_version(void) { return "zmc-gfx950 0.1"; }

}  // extern "C"
