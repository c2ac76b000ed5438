// zmc_device.hpp -- device-resident layouts shared by the host runtime and the gfx950 kernels.
//
// Work decomposition.  A function's samples are grouped in quads (4 consecutive
// samples; quad q of a d-dimensional function draws Philox blocks q*d .. q*d+d-1,
// block q*d + j holding coordinate j of the four samples) and quads in segments
// of kSegQuads = 64 lanes x kQuadsPerLane quads.  Lane l of the wave that owns
// segment s evaluates quads s*kSegQuads + k*64 + l for k = 0..15 and keeps
// compensated sums; the 64 lane sums are combined by a fixed xor butterfly in
// FP64.  Segment sums are combined by a fixed pairwise tree over the segment
// index (zero-padded to a power of two).  A tile is an aligned power-of-two run
// of segments handed to one workgroup; its sum is a subtree of that same tree,
// so a function's result is bitwise independent of the tile size, the grid
// shape, the batch it runs in and the order tiles are fetched.
#pragma once

#include <stdint.h>

namespace zmc {

constexpr int kMaxDim = 12;
constexpr int kWave = 64;
constexpr int kQuadsPerLane = 16;
constexpr int kSegQuads = kWave * kQuadsPerLane;      // 1024 quads
constexpr int kSegSamples = 4 * kSegQuads;            // 4096 samples
constexpr int kBlockWaves = 4;                        // waves per workgroup
constexpr int kBlockThreads = kWave * kBlockWaves;    // 256
constexpr int kMaxSegLog2 = 6;                        // at most 64 segments per wave per tile
constexpr int kMaxPolyDegree = 8;                     // product polynomial degrees are 0..8 (validated)
constexpr int kNumFamilies = 4;                       // built-in families
constexpr int kMaxUserFamilies = 8;                   // run-time compiled families
constexpr uint32_t kUserFamily0 = 16;                 // family id of the first run-time family
constexpr int kKernelBuiltin32 = 0;                   // kernel indices: built-in FP32, built-in FP64,
constexpr int kKernelBuiltin64 = 1;                   //   then FP32 / FP64 of each run-time family
constexpr int kMaxKernels = 2 + 2 * kMaxUserFamilies;
constexpr int kUserParams = 32;

enum Family : uint32_t { HARMONIC = 0, ABS_LINEAR = 1, GAUSSIAN = 2, POLY_PRODUCT = 3 };

// One function as the kernels read it (built on the host from mc_function).
// Everything a tile needs sits in one 64-byte-aligned record so a wave loads it
// with a handful of scalar loads.
struct alignas(64) DevFn {
    uint32_t family;
    uint32_t dim;
    uint32_t key0, key1;          // Philox key
    uint64_t n_samples;
    uint64_t n_quads;             // ceil(n_samples / 4)
    uint32_t n_segments;          // ceil(n_quads / kSegQuads)
    uint32_t precision;           // 0 = FP32 evaluation, 1 = FP64
    double volume;                // prod_j (hi_j - lo_j)
    double scale1, scale2;        // S1 = scale1 * sum g, S2 = scale2 * sum g^2 (FP32 path)

    // FP64 path: the definition, in its own operation order.
    double lo[kMaxDim];
    double w[kMaxDim];            // hi - lo
    double v[kMaxDim];            // k / c / mu / p
    double s0, s1, h;             // (a, b) / (a, c0) / (A, sigma, 0.5/sigma^2)
    int32_t deg[kMaxDim];         // POLY_PRODUCT exponents

    // FP32 path: coefficients of each family in the variable t_j = 1 + m_j 2^-23,
    // the float whose mantissa is the low 23 bits of the Philox word, so that
    // u_j = t_j - (1 - 2^-24) exactly.
    float fc[kMaxDim];            // HARMONIC kappa_j (revolutions per unit t); ABS gamma_j;
                                  // GAUSSIAN sqrt(log2(e) / (2 sigma^2)) w_j; POLY w_j
    float fo[kMaxDim];            // GAUSSIAN centre m_j in t-space; POLY lo_j
    float fp[kMaxDim];            // POLY p_j
    float f0, f0lo;               // HARMONIC phase offset (revolutions); ABS offset as hi + lo
    uint32_t kfam;                // family as the kernels dispatch on it
    uint32_t pad_;

    // Run-time compiled families: the caller's parameters as given and rounded to FP32.
    double up[kUserParams];
    float up32[kUserParams];
};

// A tile: segments [seg0, seg0 + 4 << seg_log2) of function fn (clipped to the
// function's segment count), partial written to partials[out].
struct Tile {
    uint32_t fn;
    uint32_t seg0;
    uint32_t seg_log2;            // log2 of segments per wave
    uint32_t out;
};

// Finalize record: function fn's tile partials are partials[part0 .. part0 + n_tiles).
// Consecutive tiles of one function in a launch's tile list, as the host stages
// them; the stage kernel expands each into `count` Tile records at `dst`.
struct TileRun {
    uint32_t fn;
    uint32_t first;               // the function's tile index of the first one
    uint32_t count;
    uint32_t seg_log2;
    uint32_t part0;               // partial slot of the function's tile 0
    uint32_t dst;                 // position of the first one in the tile list
    uint32_t flags;               // kRunUploadRecord: copy the function's record from the host mirror first
    uint32_t pad_;
};
constexpr uint32_t kRunUploadRecord = 1u;

struct Fin {
    uint32_t fn;
    uint32_t part0;
    uint32_t n_tiles;
    uint32_t res;                 // index into the launch's result array
};

struct Partial {
    double s1, s2;
};

// Result record, identical in layout to mc_result.
struct DevResult {
    double mean, std_error, sum_f, sum_f2;
    uint64_t n;
    int32_t status;
    uint32_t precision;
};

// Counters of one launch (zeroed by every descriptor upload).
constexpr int kCounterAborted = 0;     // a workgroup stopped because the abort word was set
constexpr int kCounterBadRecords = 1;  // tile or finalize records that failed their bounds checks
constexpr int kCounterTiles = 2;       // kMaxKernels words: next tile of each kernel
constexpr int kNumCounters = kCounterTiles + kMaxKernels;

// Everything one launch reads; lives in device memory at a fixed address per
// launch slot so a captured graph can be replayed with new contents.  The host
// writes it, with zeroed counters, the tile list and the finalize records, into
// pinned host memory; the launch's first kernel copies those `stage_bytes` into
// device memory.  The tile list is cut into one contiguous part per kernel
// (built-in FP32, built-in FP64, each run-time family in FP32 and FP64); every
// kernel walks its part and writes into the same partial arena, one finalize
// kernel turns partials into results, and a publish kernel copies results and
// counters into pinned host memory and, last, stores the launch's sequence
// number into `host_done`.
struct alignas(64) LaunchDesc {
    uint64_t stage_bytes;                  // bytes from this descriptor on that the stage kernel copies
    uint32_t n_runs;                       // tile runs staged after the finalize records
    uint32_t runs_off;                     // their byte offset from this descriptor (host block)
    const DevFn* fns;
    const Tile* tiles;
    Partial* partials;
    const Fin* fins;
    DevResult* results;                    // device: n_fins results (finalize)
    DevResult* host_results;               // host memory: their copy (publish)
    uint32_t* counters;                    // device: kNumCounters words, right after this descriptor
    uint32_t* host_counters;               // host memory: copy of the counters at the end of the launch
    uint32_t* host_done;                   // host memory: receives `seq` once results and counters are out
    const uint32_t* abort_word;            // device word; nonzero asks the kernels to stop fetching tiles
    uint64_t n_partials;                   // size of the partial arena (bounds checks)
    uint32_t n_fns;                        // size of the function table (bounds checks)
    uint32_t n_fins;
    uint32_t seq;
    uint32_t pad_;
    uint32_t tile_begin[kMaxKernels];
    uint32_t tile_count[kMaxKernels];
};

// ---------------------------------------------------------------- resident engine
//
// A context created with MC_RESIDENT keeps one persistent kernel on the GPU
// while work keeps coming.  The host appends chunks -- up to kChunkTiles
// consecutive tiles of one function -- to a ring in pinned, fine-grained host
// memory and publishes the count in a control word.  A workgroup takes a
// ticket (an atomic add on a device counter) and processes ring entry
// `ticket` once the control word shows it; the workgroup that counts a
// function's last tile reduces its partials with the finalize tree, writes the
// result into pinned host memory and then stores the run's token into the
// slot's done word the host polls.  Nothing is launched per batch of work.
//
// Records are read through the scalar cache, which is only invalidated when a
// kernel starts, so a record address is never written twice within one launch:
// every run gets a fresh position in a record arena (its first chunk copies the
// record there from the host mirror), and the host relaunches the kernel before
// it reuses a position read in the current launch.
//
// Stopping.  The control word's top bit asks workgroups to leave; once it is
// set (by the host, or by a workgroup that waited `idle_polls` times for its
// ticket) the device's copy of the word never changes again, so every
// workgroup sees the same final count: tickets below it are processed, the rest
// are left, and the processed entries are exactly a prefix of the ring that
// the host finds from the entries' acknowledgement words.
constexpr uint32_t kChunkTiles = 8;
constexpr uint32_t kChunkUpload = 1u;         // copy the record from the host mirror into the arena first
constexpr uint64_t kCtlStop = 1ull << 63;     // in the control word: leave

struct Chunk {
    uint32_t fn;                  // function slot (counters, result and done word)
    uint32_t rec;                 // record arena position of this run
    uint32_t first;               // the function's tile index of the first tile
    uint32_t count;               // tiles, 1..kChunkTiles
    uint32_t part0;               // partial slot of the function's tile 0
    uint32_t n_tiles;             // the run's tiles (its result is out when all are counted)
    uint32_t token;               // nonzero, unique per run: reported in the done word
    uint32_t seg_flags;           // seg_log2 in bits 0..7, kChunkUpload << 8
};

struct alignas(64) ResidentDesc {
    const Chunk* ring;            // host: ring_mask + 1 entries
    uint64_t* ack;                // host: per entry, its position + 1 once a workgroup has read it
    const uint64_t* host_ctl;     // host: entries written (bits 0..62), kCtlStop
    uint32_t* host_exit;          // host: the launch's epoch, stored by the last workgroup to leave;
                                  // the word after it receives the bad-chunk count first
    DevResult* host_results;      // host: per function slot
    uint32_t* host_done;          // host: per function slot, the token of the run whose result is out
    const DevFn* mirror;          // host: packed records by function slot
    DevFn* arena;                 // device: record arena
    Partial* partials;
    uint64_t* pos;                // device: [0] tickets issued, [1] control word as last seen (top bit: stop)
    uint32_t* running;            // device: workgroups of the launch not yet gone
    uint32_t* tiles_done;         // device: per function slot, tiles counted in the current run
    uint32_t* ready;              // device: per arena position, token of the run whose record is in place
    uint32_t* slot_err;           // device: per function slot, token of a run that met a bad chunk or a timeout
    uint32_t* bad_records;        // device: chunks that failed their checks
    uint64_t n_partials;
    uint32_t n_fns;
    uint32_t n_arena;
    uint32_t ring_mask;
    uint32_t idle_polls;          // polls for a ticket's entry before the workgroup stops the launch
    uint32_t ready_polls;         // polls of a record's ready word before the chunk is given up
    uint32_t leader_every;        // workgroups with blockIdx % leader_every == 0 read the host's control word
};

}  // namespace zmc
