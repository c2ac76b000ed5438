// emu_scenarios.cpp -- the library's host runtime driven through its C ABI on
// the CPU emulation of HIP (test infrastructure only; see hipemu.cpp).
//
// Usage: emu_scenarios <scenario> ...   (or "all").  Prints "ok <scenario>" per
// passing scenario; exits non-zero on the first failure.  Every result the
// library reports as MC_OK is compared field by field with the result the
// emulation defines for that function (hipemu::expected_batched / plain).
#include <unistd.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "hipemu.hpp"
#include "zmc.h"
#include <hip/hip_runtime.h>  // (the emulation's: host/device keywords for the packing header)

#include "zmc_pack.hpp"

namespace {

int g_failures = 0;

#define CHECK(cond, ...)                                                          \
    do {                                                                          \
        if (!(cond)) {                                                            \
            std::fprintf(stderr, "%s:%d: check failed: %s: ", __FILE__, __LINE__, #cond); \
            std::fprintf(stderr, __VA_ARGS__);                                    \
            std::fprintf(stderr, "\n");                                           \
            ++g_failures;                                                         \
            return false;                                                         \
        }                                                                         \
    } while (0)

// A function of one of the built-in families on a box, amplitude 1 unless given.
mc_function make_fn(uint32_t family, uint32_t dim, uint64_t n, uint64_t seed, double amp = 1.0)
{
    mc_function f;
    std::memset(&f, 0, sizeof f);
    f.family = family;
    f.dim = dim;
    f.n_samples = n;
    f.seed = seed;
    for (uint32_t j = 0; j < dim; ++j) {
        f.lo[j] = -0.5 + 0.1 * j;
        f.hi[j] = f.lo[j] + 1.0 + 0.05 * j;
    }
    f.params[0] = amp;
    switch (family) {
    case MC_FAMILY_HARMONIC:
        f.params[1] = 0.0;
        for (uint32_t j = 0; j < dim; ++j) f.params[MC_PARAM_V0 + j] = 2.0 + j;
        break;
    case MC_FAMILY_ABS_LINEAR:
        f.params[1] = 0.25;
        for (uint32_t j = 0; j < dim; ++j) f.params[MC_PARAM_V0 + j] = (j & 1) ? -1.0 : 1.0;
        break;
    case MC_FAMILY_GAUSSIAN:
        f.params[1] = 0.5;
        for (uint32_t j = 0; j < dim; ++j) f.params[MC_PARAM_V0 + j] = 0.1;
        break;
    default:
        f.params[0] = 0.0;
        for (uint32_t j = 0; j < dim; ++j) {
            f.params[MC_PARAM_V0 + j] = 0.5;
            f.params[MC_PARAM_W0 + j] = 1 + j % 4;
        }
        break;
    }
    return f;
}

// A mixed table: every family, dimensions 1..12, sizes from 2 samples to several
// segments and tiles with ragged tails.  Rows with `constant_every` > 0 and
// index % constant_every == 1 have seed bit 63 set (constant in the emulated
// FP32 kernel, so an FP32 request promotes them).
std::vector<mc_function> mixed_table(size_t n, uint64_t base, size_t constant_every = 0)
{
    static const uint64_t sizes[] = {2, 3, 5, 64, 4095, 4096, 4097, 16385, 70001, 300003, 1000001};
    std::vector<mc_function> t;
    for (size_t i = 0; i < n; ++i) {
        uint64_t seed = (base << 32) | i;
        if (constant_every && i % constant_every == 1) seed |= 1ull << 63;
        t.push_back(make_fn((uint32_t)(i % 4), 1 + (uint32_t)(i % 12), sizes[(i * 7) % 11], seed));
    }
    return t;
}

bool same_result(const mc_result& a, const mc_result& b)
{
    return std::memcmp(&a, &b, sizeof a) == 0;
}

// Results of an FP32 (fp64 = false) or FP64 request against the emulation's values.
bool check_results(const std::vector<mc_function>& t, const std::vector<mc_result>& r, bool fp64, const char* label)
{
    CHECK(t.size() == r.size(), "%s: sizes", label);
    for (size_t i = 0; i < t.size(); ++i) {
        const bool promoted = !fp64 && (t[i].seed >> 63) != 0;
        const mc_result want = hipemu::expected_batched(t[i], fp64 || promoted);
        CHECK(same_result(r[i], want), "%s: function %zu: got (%.17g, %.17g, %.17g, n %llu, status %d, prec %u) "
              "want (%.17g, %.17g, %.17g, prec %u)", label, i, r[i].mean, r[i].sum_f, r[i].sum_f2,
              (unsigned long long)r[i].n, r[i].status, r[i].precision, want.mean, want.sum_f, want.sum_f2,
              want.precision);
    }
    return true;
}

mc_ctx* create(uint32_t flags, uint32_t max_tiles = 0, uint32_t policy = MC_SCHED_FAIR, uint32_t max_functions = 0,
               uint64_t max_partials = 0)
{
    mc_config cfg;
    mc_config_init(&cfg);
    cfg.flags = flags;
    cfg.max_tiles_per_run = max_tiles;
    cfg.policy = policy;
    cfg.max_functions = max_functions;
    cfg.max_partials = max_partials;
    mc_ctx* ctx = nullptr;
    if (mc_create(&cfg, &ctx) != MC_OK) return nullptr;
    return ctx;
}

// Results of a request that was aborted or cancelled: those that came in are exact,
// the others carry MC_ERR_ABORTED.
bool check_cancelled(const std::vector<mc_function>& t, const std::vector<mc_result>& r, const char* label,
                     bool fp64 = false)
{
    for (size_t i = 0; i < t.size(); ++i) {
        if (r[i].status == MC_OK) {
            const bool promoted = !fp64 && (t[i].seed >> 63) != 0;
            const mc_result want = hipemu::expected_batched(t[i], fp64 || promoted);
            CHECK(same_result(r[i], want), "%s: function %zu kept a wrong result: got (%.17g, n %llu, prec %u) want "
                  "(%.17g, n %llu, prec %u)", label, i, r[i].mean, (unsigned long long)r[i].n, r[i].precision,
                  want.mean, (unsigned long long)want.n, want.precision);
        } else {
            CHECK(r[i].status == MC_ERR_ABORTED && r[i].n == t[i].n_samples, "%s: function %zu: status %d", label, i,
                  r[i].status);
        }
    }
    return true;
}

bool run_request(mc_ctx* ctx, const std::vector<mc_function>& t, bool fp64, const char* label)
{
    uint64_t id = 0;
    CHECK(mc_submit(ctx, t.data(), t.size(), fp64 ? MC_PREC_FP64 : MC_PREC_FP32_EVAL, &id) == MC_OK, "%s: %s", label,
          mc_last_error(ctx));
    std::vector<mc_result> r(t.size());
    CHECK(mc_results(ctx, id, r.data(), r.size(), 1) == MC_OK, "%s: %s", label, mc_last_error(ctx));
    return check_results(t, r, fp64, label);
}

// ---------------------------------------------------------------- scenarios

bool basic()
{
    for (uint32_t flags : {0u, (uint32_t)MC_NO_GRAPH}) {
        mc_ctx* ctx = create(flags);
        CHECK(ctx, "create");
        const std::vector<mc_function> t = mixed_table(60, 1, 7);
        if (!run_request(ctx, t, false, "fp32") || !run_request(ctx, t, true, "fp64")) return false;
        mc_stats st;
        CHECK(mc_get_stats(ctx, &st) == MC_OK && st.bad_records == 0, "stats");
        CHECK(st.promoted == 9, "promoted %llu", (unsigned long long)st.promoted);
        mc_destroy(ctx);
    }
    return true;
}

// Launches of a few tiles each: functions span many launches, under every policy.
bool many_launches()
{
    for (uint32_t policy : {MC_SCHED_FAIR, MC_SCHED_FIFO, MC_SCHED_SRPT})
        for (uint32_t flags : {0u, (uint32_t)MC_NO_GRAPH}) {
            mc_ctx* ctx = create(flags, 5, policy);
            CHECK(ctx, "create");
            std::vector<std::vector<mc_function>> reqs = {mixed_table(12, 2, 5), mixed_table(3, 3), mixed_table(30, 4)};
            std::vector<uint64_t> ids;
            for (size_t k = 0; k < reqs.size(); ++k) {
                uint64_t id = 0;
                CHECK(mc_submit(ctx, reqs[k].data(), reqs[k].size(), k == 1 ? MC_PREC_FP64 : MC_PREC_FP32_EVAL, &id) ==
                          MC_OK, "submit");
                ids.push_back(id);
            }
            // drive with mc_run / mc_poll only, as a serving loop would
            std::map<uint64_t, bool> done;
            for (int guard = 0; guard < 100000 && done.size() < ids.size(); ++guard) {
                const mc_status st = mc_run(ctx, nullptr);
                CHECK(st == MC_OK || st == MC_NOT_READY, "run %d: %s", (int)st, mc_last_error(ctx));
                uint64_t got[8];
                size_t n = 0;
                CHECK(mc_poll(ctx, got, 8, &n) == MC_OK, "poll");
                for (size_t i = 0; i < n; ++i) done[got[i]] = true;
            }
            CHECK(done.size() == ids.size(), "requests did not all complete");
            for (size_t k = 0; k < reqs.size(); ++k) {
                std::vector<mc_result> r(reqs[k].size());
                CHECK(mc_results(ctx, ids[k], r.data(), r.size(), 0) == MC_OK, "results");
                if (!check_results(reqs[k], r, k == 1, "many launches")) return false;
            }
            uint64_t pr = 1, pt = 1;
            CHECK(mc_pending(ctx, &pr, &pt) == MC_OK && pr == 0 && pt == 0, "pending %llu %llu", (unsigned long long)pr,
                  (unsigned long long)pt);
            mc_destroy(ctx);
        }
    return true;
}

// Requests wait for function slots and partial space; ones that never fit are refused.
bool admission()
{
    mc_ctx* ctx = create(0, 64, MC_SCHED_FIFO, 16, 400);  // one request of 10 at a time
    CHECK(ctx, "create");
    std::vector<std::vector<mc_function>> reqs;
    std::vector<uint64_t> ids;
    for (int k = 0; k < 6; ++k) {
        reqs.push_back(mixed_table(10, 10 + k));
        uint64_t id = 0;
        CHECK(mc_submit(ctx, reqs.back().data(), 10, MC_PREC_FP32_EVAL, &id) == MC_OK, "submit %d: %s", k,
              mc_last_error(ctx));
        ids.push_back(id);
    }
    uint64_t id = 0;
    const std::vector<mc_function> big = mixed_table(17, 30);
    CHECK(mc_submit(ctx, big.data(), big.size(), MC_PREC_FP32_EVAL, &id) == MC_ERR_ADMISSION, "17 functions");
    std::vector<mc_function> wide(1, make_fn(MC_FAMILY_HARMONIC, 3, 401ull * 4 * 4096, 5));  // 401 tiles of 4 segments
    CHECK(mc_submit(ctx, wide.data(), 1, MC_PREC_FP32_EVAL, &id) == MC_ERR_ADMISSION, "401 partials");
    for (size_t k = ids.size(); k-- > 0;) {  // newest first: blocking calls drive the queue
        std::vector<mc_result> r(10);
        CHECK(mc_results(ctx, ids[k], r.data(), 10, 1) == MC_OK, "results %zu: %s", k, mc_last_error(ctx));
        if (!check_results(reqs[k], r, false, "admission")) return false;
    }
    mc_destroy(ctx);
    return true;
}

bool grid()
{
    mc_ctx* ctx = create(0, 9);
    CHECK(ctx, "create");
    const mc_function base = make_fn(MC_FAMILY_HARMONIC, 3, 50001, 7ull << 32, 1.5);
    mc_grid_axis axes[2] = {{MC_PARAM_V0, 5, 1.0, 0.5}, {0, 3, 0.5, 0.25}};
    for (int prec : {MC_PREC_FP32_EVAL, MC_PREC_FP64}) {
        uint64_t id = 0;
        CHECK(mc_submit_grid(ctx, &base, axes, 2, prec, &id) == MC_OK, "grid: %s", mc_last_error(ctx));
        std::vector<mc_result> r(15);
        CHECK(mc_results(ctx, id, r.data(), 15, 1) == MC_OK, "grid results");
        std::vector<mc_function> t;
        for (uint64_t i = 0; i < 15; ++i) {
            mc_function f = base;
            f.params[MC_PARAM_V0] = 1.0 + (double)(i % 5) * 0.5;
            f.params[0] = 0.5 + (double)(i / 5) * 0.25;
            f.seed = base.seed + i;
            t.push_back(f);
        }
        if (!check_results(t, r, prec == MC_PREC_FP64, "grid")) return false;
    }
    mc_destroy(ctx);
    return true;
}

bool abort_and_continue()
{
    mc_ctx* ctx = create(MC_NO_GRAPH, 4);
    CHECK(ctx, "create");
    const std::vector<mc_function> t = mixed_table(24, 40);
    uint64_t id = 0;
    CHECK(mc_submit(ctx, t.data(), t.size(), MC_PREC_FP32_EVAL, &id) == MC_OK, "submit");
    CHECK(mc_run(ctx, nullptr) == MC_OK, "run");
    CHECK(mc_abort(ctx) == MC_OK, "abort");
    uint64_t later = 0;  // submitted after the abort call, before the step that carries it out
    const std::vector<mc_function> t2 = mixed_table(6, 42);
    CHECK(mc_submit(ctx, t2.data(), t2.size(), MC_PREC_FP32_EVAL, &later) == MC_OK, "submit after the abort");
    std::vector<mc_result> r(t.size());
    CHECK(mc_results(ctx, id, r.data(), r.size(), 1) == MC_ERR_ABORTED, "aborted request");
    size_t ok = 0;
    for (size_t i = 0; i < t.size(); ++i) {
        if (r[i].status == MC_OK) {
            ++ok;
            CHECK(same_result(r[i], hipemu::expected_batched(t[i], false)), "finished before the abort: %zu", i);
        } else {
            CHECK(r[i].status == MC_ERR_ABORTED, "status %d", r[i].status);
        }
    }
    CHECK(ok < t.size(), "nothing was aborted");
    std::vector<mc_result> r2(t2.size());
    CHECK(mc_results(ctx, later, r2.data(), r2.size(), 1) == MC_OK, "submitted after the abort: %s", mc_last_error(ctx));
    if (!check_results(t2, r2, false, "submitted after the abort")) return false;
    if (!run_request(ctx, mixed_table(8, 41), false, "after abort")) return false;
    mc_destroy(ctx);
    return true;
}

bool errors()
{
    mc_ctx* ctx = create(0);
    CHECK(ctx, "create");
    std::vector<mc_function> t = mixed_table(5, 50);
    uint64_t id = 0;
    struct Bad {
        int field;
        mc_status code;
    } bads[] = {{0, MC_ERR_BAD_DIM}, {1, MC_ERR_BAD_BOUNDS}, {2, MC_ERR_BAD_PARAMS}, {3, MC_ERR_INVALID_ARG},
                {4, MC_ERR_UNSUPPORTED_FAMILY}};
    for (const Bad& b : bads) {
        std::vector<mc_function> u = t;
        switch (b.field) {
        case 0: u[3].dim = 13; break;
        case 1: u[3].hi[0] = u[3].lo[0]; break;
        case 2: u[3].params[20] = NAN; break;
        case 3: u[3].n_samples = 1; break;
        default: u[3].family = 9; break;
        }
        CHECK(mc_submit(ctx, u.data(), u.size(), MC_PREC_FP32_EVAL, &id) == b.code, "invalid field %d", b.field);
        CHECK(std::strstr(mc_last_error(ctx), "function 3") != nullptr, "message names the row: %s", mc_last_error(ctx));
    }
    CHECK(mc_submit(ctx, t.data(), t.size(), 7, &id) == MC_ERR_INVALID_ARG, "precision");
    CHECK(mc_submit(ctx, t.data(), 0, MC_PREC_FP64, &id) == MC_ERR_INVALID_ARG, "empty");
    std::vector<mc_result> r(t.size());
    CHECK(mc_results(ctx, 12345, r.data(), r.size(), 1) == MC_ERR_UNKNOWN_REQUEST, "unknown id");
    CHECK(mc_submit(ctx, t.data(), t.size(), MC_PREC_FP64, &id) == MC_OK, "submit");
    CHECK(mc_results(ctx, id, r.data(), r.size() - 1, 1) == MC_ERR_INVALID_ARG, "wrong n");
    CHECK(mc_results(ctx, id, r.data(), r.size(), 1) == MC_OK, "results");
    CHECK(mc_results(ctx, id, r.data(), r.size(), 1) == MC_ERR_UNKNOWN_REQUEST, "taken twice");
    uint32_t fam = 0;
    CHECK(mc_register_family(ctx, "template <class T> __device__ T mc_user_integrand(const T*, const T*, uint32_t)"
                                  " { return T(1); }", &fam) == MC_ERR_COMPILE, "no compiler in the emulation");
    mc_destroy(ctx);
    mc_config cfg;
    mc_config_init(&cfg);
    cfg.policy = 3;
    mc_ctx* bad = nullptr;
    CHECK(mc_create(&cfg, &bad) == MC_ERR_INVALID_ARG && bad == nullptr, "policy");
    mc_ctx* v = create(MC_VALIDATE_ONLY);
    CHECK(v, "validate-only");
    CHECK(mc_submit(v, t.data(), t.size(), MC_PREC_FP32_EVAL, &id) == MC_OK, "validate-only submit");
    CHECK(mc_run(v, nullptr) == MC_ERR_NO_DEVICE, "validate-only run");
    mc_destroy(v);
    return true;
}

bool plain_paths()
{
    mc_ctx* ctx = create(0);
    CHECK(ctx, "create");
    for (size_t n : {40, 7}) {  // a smaller table second: the fixed array keeps the first call's contents
        const std::vector<mc_function> t = mixed_table(n, 60 + n);
        std::vector<mc_result> a(n), b(n);
        CHECK(mc_integrate_plain_fp64(ctx, t.data(), n, a.data(), nullptr) == MC_OK, "plain: %s", mc_last_error(ctx));
        CHECK(mc_integrate_plain_fp64_noalloc(ctx, t.data(), n, b.data(), nullptr) == MC_OK, "noalloc: %s",
              mc_last_error(ctx));
        for (size_t i = 0; i < n; ++i) {
            const mc_result want = hipemu::expected_plain(t[i]);
            CHECK(same_result(a[i], want) && same_result(b[i], want), "plain function %zu", i);
        }
    }
    std::vector<mc_function> over(4097, make_fn(MC_FAMILY_HARMONIC, 1, 10, 1));
    std::vector<mc_result> r(4097);
    CHECK(mc_integrate_plain_fp64_noalloc(ctx, over.data(), over.size(), r.data(), nullptr) == MC_ERR_INVALID_ARG,
          "4097 functions");
    over.resize(2);
    over[1].n_samples = (1ull << 30) + 1;
    CHECK(mc_integrate_plain_fp64_noalloc(ctx, over.data(), 2, r.data(), nullptr) == MC_ERR_INVALID_ARG, "2^30 + 1");
    mc_destroy(ctx);
    return true;
}

bool two_contexts()
{
    mc_ctx* a = create(0, 6);
    mc_ctx* b = create(MC_NO_GRAPH, 11, MC_SCHED_SRPT);
    CHECK(a && b, "create");
    const std::vector<mc_function> ta = mixed_table(20, 70), tb = mixed_table(25, 71, 3);
    uint64_t ia = 0, ib = 0;
    CHECK(mc_submit(a, ta.data(), ta.size(), MC_PREC_FP32_EVAL, &ia) == MC_OK, "submit a");
    CHECK(mc_submit(b, tb.data(), tb.size(), MC_PREC_FP32_EVAL, &ib) == MC_OK, "submit b");
    for (int i = 0; i < 3; ++i) {
        CHECK(mc_run(a, nullptr) != MC_ERR_HIP && mc_run(b, nullptr) != MC_ERR_HIP, "run");
    }
    std::vector<mc_result> ra(ta.size()), rb(tb.size());
    CHECK(mc_results(b, ib, rb.data(), rb.size(), 1) == MC_OK, "b");
    CHECK(mc_results(a, ia, ra.data(), ra.size(), 1) == MC_OK, "a");
    if (!check_results(ta, ra, false, "context a") || !check_results(tb, rb, false, "context b")) return false;
    mc_destroy(a);
    mc_destroy(b);
    return true;
}

// One run of the failure-injection workload: three requests (FP32 with promoted
// rows, FP64, a grid) in launches of a few tiles, driven by mc_run and
// non-blocking mc_results.  Every call may fail; a request that returns MC_OK
// must hold exactly the expected results, every other one must end with
// MC_ERR_HIP or MC_ERR_OUT_OF_MEMORY.  *clean: nothing failed.
bool fault_workload(uint32_t flags, bool* clean)
{
    *clean = true;
    mc_ctx* ctx = create(flags, 6, MC_SCHED_FAIR, 64, 4096);
    if (!ctx) {
        *clean = false;
        const std::string e = mc_last_error(nullptr);
        CHECK(e.find("failed") != std::string::npos, "create failed without a message");
        return true;
    }
    std::vector<std::vector<mc_function>> reqs = {mixed_table(14, 80, 4), mixed_table(5, 81)};
    const mc_function base = make_fn(MC_FAMILY_GAUSSIAN, 2, 9001, 82ull << 32);
    mc_grid_axis axis = {MC_PARAM_V0, 4, 0.0, 0.25};
    std::vector<mc_function> grid_t;
    for (uint64_t i = 0; i < 4; ++i) {
        mc_function f = base;
        f.params[MC_PARAM_V0] = (double)i * 0.25;
        f.seed = base.seed + i;
        grid_t.push_back(f);
    }
    // request 3 is cancelled after the first run; requests 4 and 5 are
    // request 0, snapshotted then and restored into the same context, and 5
    // is cancelled after the second run
    reqs.push_back(grid_t);
    reqs.push_back(mixed_table(9, 83));
    reqs.push_back(reqs[0]);
    reqs.push_back(reqs[0]);
    std::vector<uint64_t> ids(6, 0);
    std::vector<int> state(6, 0);  // 0 not submitted, 1 pending, 2 done
    state[4] = state[5] = 2;
    for (int k = 0; k < 4; ++k) {
        mc_status st = k == 2 ? mc_submit_grid(ctx, &base, &axis, 1, MC_PREC_FP32_EVAL, &ids[k])
                              : mc_submit(ctx, reqs[k].data(), reqs[k].size(), k == 1 ? MC_PREC_FP64 : MC_PREC_FP32_EVAL,
                                          &ids[k]);
        if (st == MC_OK) {
            state[k] = 1;
        } else {
            *clean = false;
            CHECK(st == MC_ERR_HIP || st == MC_ERR_OUT_OF_MEMORY, "submit %d: status %d", k, (int)st);
            state[k] = 2;
        }
    }
    for (int guard = 0; guard < 20000; ++guard) {
        bool all = true;
        for (int k = 0; k < 6; ++k) all = all && state[k] == 2;
        if (all) break;
        const mc_status st = mc_run(ctx, nullptr);
        if (st != MC_OK && st != MC_NOT_READY) {
            *clean = false;
            CHECK(st == MC_ERR_HIP || st == MC_ERR_OUT_OF_MEMORY, "run: status %d", (int)st);
        }
        if (guard == 0 && state[3] == 1) {
            const mc_status cs = mc_cancel(ctx, ids[3]);
            if (cs != MC_OK) {
                *clean = false;
                CHECK(cs == MC_ERR_HIP, "cancel: status %d", (int)cs);
            }
        }
        if (guard == 0 && state[0] == 1) {
            size_t need = 0, got = 0;
            std::vector<uint8_t> blob;
            mc_status ss = mc_snapshot(ctx, ids[0], nullptr, 0, &need);
            if (ss == MC_OK) {
                blob.resize(need);
                ss = mc_snapshot(ctx, ids[0], blob.data(), blob.size(), &got);
            }
            if (ss == MC_OK) ss = mc_restore(ctx, blob.data(), got, &ids[4]);
            if (ss == MC_OK) state[4] = 1;
            if (ss == MC_OK) ss = mc_restore(ctx, blob.data(), got, &ids[5]);
            if (ss == MC_OK) {
                state[5] = 1;
            } else {
                // (a request lost with a failed launch cannot be snapshotted)
                *clean = false;
                const std::string e = mc_last_error(ctx);
                CHECK(ss == MC_ERR_HIP || ss == MC_ERR_OUT_OF_MEMORY ||
                          (ss == MC_ERR_INVALID_ARG && e.find("aborted or failed") != std::string::npos),
                      "snapshot and restore: status %d: %s", (int)ss, e.c_str());
            }
        }
        if (guard == 1 && state[5] == 1) {
            const mc_status cs = mc_cancel(ctx, ids[5]);
            if (cs != MC_OK) {
                *clean = false;
                CHECK(cs == MC_ERR_HIP, "cancel of the restored copy: status %d", (int)cs);
            }
        }
        for (int k = 0; k < 6; ++k) {
            if (state[k] != 1) continue;
            const std::vector<mc_function>& t = reqs[k];
            std::vector<mc_result> r(t.size());
            const mc_status rs = mc_results(ctx, ids[k], r.data(), r.size(), guard > 10000);
            if (rs == MC_NOT_READY) continue;
            state[k] = 2;
            if (rs == MC_OK) {
                // (the cancelled request too, if the cancel failed before it took effect)
                if (!check_results(t, r, k == 1, k == 4 ? "restored copy, after injected failures" : "after injected failures"))
                    return false;
            } else if (rs == MC_ERR_ABORTED && (k == 3 || k == 5)) {
                if (!check_cancelled(t, r, "cancelled")) return false;
            } else {
                *clean = false;
                CHECK(rs == MC_ERR_HIP || rs == MC_ERR_OUT_OF_MEMORY, "results %d: status %d", k, (int)rs);
            }
        }
    }
    for (int k = 0; k < 6; ++k) CHECK(state[k] == 2, "request %d never finished", k);
    // the context still works: a new request completes (the injected failure
    // fires once, so if it lands here the second attempt must succeed)
    const std::vector<mc_function> after = mixed_table(6, 83);
    bool done = false;
    for (int attempt = 0; attempt < 2 && !done; ++attempt) {
        uint64_t id = 0;
        mc_status rs = mc_submit(ctx, after.data(), after.size(), MC_PREC_FP32_EVAL, &id);
        std::vector<mc_result> r(after.size());
        if (rs == MC_OK) rs = mc_results(ctx, id, r.data(), r.size(), 1);
        if (rs == MC_OK) {
            if (!check_results(after, r, false, "after the failures")) return false;
            done = true;
        } else {
            *clean = false;
            CHECK(attempt == 0 && (rs == MC_ERR_HIP || rs == MC_ERR_OUT_OF_MEMORY),
                  "a request after the failures: status %d: %s", (int)rs, mc_last_error(ctx));
            if (id != 0) mc_results(ctx, id, r.data(), r.size(), 1);  // release it if it is still queued
        }
    }
    CHECK(done, "no request completed after the failures");
    mc_destroy(ctx);
    return true;
}

// Fail the n-th checked HIP call, for every n the workload makes, with and
// without graphs, and on a resident context.
bool fault_sweep()
{
    for (uint32_t flags : {(uint32_t)MC_NO_GRAPH, 0u, (uint32_t)MC_RESIDENT}) {
        unsetenv("MC_FAULT_HIP");
        bool clean = false;
        const uint64_t c0 = hipemu::api_calls();
        if (!fault_workload(flags, &clean)) return false;
        CHECK(clean, "the workload fails without injected failures");
        const int calls = (int)(hipemu::api_calls() - c0);
        int failed_runs = 0;
        for (int n = 1; n <= calls + 2; ++n) {
            char buf[32];
            std::snprintf(buf, sizeof buf, "%d", n);
            setenv("MC_FAULT_HIP", buf, 1);
            clean = true;
            if (!fault_workload(flags, &clean)) {
                std::fprintf(stderr, "fault sweep: failing call %d (flags %u)\n", n, flags);
                unsetenv("MC_FAULT_HIP");
                return false;
            }
            failed_runs += clean ? 0 : 1;
        }
        unsetenv("MC_FAULT_HIP");
        CHECK(failed_runs > calls / 4, "only %d of %d runs saw a failure", failed_runs, calls + 2);
        std::printf("fault sweep (flags %u): each of the first %d checked HIP calls failed in turn; %d runs saw an "
                    "error\n", flags, calls + 2, failed_runs);
    }
    return true;
}

// The tuning cache: a tuned context appends its choice to MC_TUNE_CACHE; a new
// context on the same device kind takes the cached line (the last matching one)
// instead of timing again; malformed or foreign lines are ignored; results do
// not depend on the tuning.
bool autotune_cache()
{
    char path[] = "/tmp/zmc_tune_XXXXXX";
    const int fd = mkstemp(path);
    CHECK(fd >= 0, "mkstemp");
    close(fd);
    setenv("MC_TUNE_CACHE", path, 1);
    bool ok = [&]() -> bool {
        mc_ctx* a = create(0);
        CHECK(a, "create");
        const std::vector<mc_function> t = mixed_table(20, 90);
        uint64_t id = 0;
        std::vector<mc_result> before(t.size()), after(t.size());
        CHECK(mc_submit(a, t.data(), t.size(), MC_PREC_FP32_EVAL, &id) == MC_OK, "submit");
        CHECK(mc_results(a, id, before.data(), before.size(), 1) == MC_OK, "results");
        CHECK(mc_autotune(a, MC_PREC_FP32_EVAL, nullptr, 0.5) == MC_OK, "autotune: %s", mc_last_error(a));
        CHECK(mc_submit(a, t.data(), t.size(), MC_PREC_FP32_EVAL, &id) == MC_OK, "submit");
        CHECK(mc_results(a, id, after.data(), after.size(), 1) == MC_OK, "results");
        for (size_t i = 0; i < t.size(); ++i) CHECK(same_result(before[i], after[i]), "result %zu changed", i);
        mc_destroy(a);
        // the cache holds one line; rewrite its values, add noise around it
        FILE* f = std::fopen(path, "r");
        CHECK(f, "cache file");
        char line[2048] = {};
        CHECK(std::fgets(line, sizeof line, f) != nullptr, "cache line");
        char extra[16];
        CHECK(std::fgets(extra, sizeof extra, f) == nullptr, "one line");
        std::fclose(f);
        std::string l(line);
        size_t pos = 0;
        for (int field = 0; field < 7; ++field) pos = l.find(' ', pos) + 1;  // up to "<blocks per CU>"
        std::string edited = l.substr(0, pos) + "3";
        for (int i = 0; i < 96; ++i) edited += i < 48 ? " 2" : " 1";
        f = std::fopen(path, "w");
        std::fputs("garbage line\n", f);
        std::fputs((l.substr(0, pos) + "99 1 2 3\n").c_str(), f);  // blocks out of range: ignored
        std::fputs((edited + "\n").c_str(), f);
        std::fputs("zmc-tune 1 gfx000 8 other 0 5 0 0\n", f);     // another device: ignored
        std::fclose(f);
        mc_ctx* b = create(0);
        CHECK(b, "create");
        uint32_t blocks = 0;
        uint8_t defaults[96], seg[96];
        CHECK(mc_get_tuning(b, &blocks, defaults) == MC_OK, "default tuning");
        CHECK(mc_autotune(b, MC_PREC_FP32_EVAL, nullptr, 0.5) == MC_OK, "cached autotune");
        CHECK(mc_get_tuning(b, &blocks, seg) == MC_OK, "get tuning");
        CHECK(blocks == 3, "blocks per CU from the cache: %u", blocks);
        // FP32 rows from the cache, the FP64 rows untouched
        for (int i = 0; i < 96; ++i) CHECK(seg[i] == (i < 48 ? 2 : defaults[i]), "seg %d = %u", i, (unsigned)seg[i]);
        mc_destroy(b);
        return true;
    }();
    unsetenv("MC_TUNE_CACHE");
    std::remove(path);
    return ok;
}

// ---------------------------------------------------------------- resident contexts

// Drive requests with mc_run / mc_poll only; returns the ids in completion order.
bool drive(mc_ctx* ctx, size_t n_requests, std::vector<uint64_t>* order, int max_steps = 2000000)
{
    for (int guard = 0; guard < max_steps && order->size() < n_requests; ++guard) {
        const mc_status st = mc_run(ctx, nullptr);
        CHECK(st == MC_OK, "run %d: %s", (int)st, mc_last_error(ctx));
        uint64_t got[16];
        size_t n = 0;
        CHECK(mc_poll(ctx, got, 16, &n) == MC_OK, "poll");
        for (size_t i = 0; i < n; ++i) order->push_back(got[i]);
    }
    CHECK(order->size() == n_requests, "%zu of %zu requests completed", order->size(), n_requests);
    return true;
}

// Every policy: FP32 requests with rows the FP32 check sends to FP64 (a second
// run of the function, with a new record), FP64 requests and a grid, submitted
// together and served by the resident kernel; results exactly as the launch
// path gives them; nothing left pending; a launch context beside it agrees.
bool resident_basic()
{
    for (uint32_t policy : {MC_SCHED_FAIR, MC_SCHED_FIFO, MC_SCHED_SRPT}) {
        mc_ctx* ctx = create(MC_RESIDENT, 0, policy);
        CHECK(ctx, "create: %s", mc_last_error(nullptr));
        std::vector<std::vector<mc_function>> reqs = {mixed_table(40, 100, 7), mixed_table(3, 101), mixed_table(60, 102),
                                                      mixed_table(25, 103, 5)};
        std::vector<uint64_t> ids;
        for (size_t k = 0; k < reqs.size(); ++k) {
            uint64_t id = 0;
            CHECK(mc_submit(ctx, reqs[k].data(), reqs[k].size(), k == 1 ? MC_PREC_FP64 : MC_PREC_FP32_EVAL, &id) ==
                      MC_OK, "submit: %s", mc_last_error(ctx));
            ids.push_back(id);
        }
        const mc_function base = make_fn(MC_FAMILY_HARMONIC, 3, 50001, 7ull << 32, 1.5);
        mc_grid_axis axes[2] = {{MC_PARAM_V0, 5, 1.0, 0.5}, {0, 3, 0.5, 0.25}};
        uint64_t gid = 0;
        CHECK(mc_submit_grid(ctx, &base, axes, 2, MC_PREC_FP32_EVAL, &gid) == MC_OK, "grid: %s", mc_last_error(ctx));
        std::vector<uint64_t> order;
        if (!drive(ctx, ids.size() + 1, &order)) return false;
        for (size_t k = 0; k < reqs.size(); ++k) {
            std::vector<mc_result> r(reqs[k].size());
            CHECK(mc_results(ctx, ids[k], r.data(), r.size(), 0) == MC_OK, "results: %s", mc_last_error(ctx));
            if (!check_results(reqs[k], r, k == 1, "resident")) return false;
        }
        std::vector<mc_result> gr(15);
        CHECK(mc_results(ctx, gid, gr.data(), 15, 0) == MC_OK, "grid results");
        std::vector<mc_function> gt;
        for (uint64_t i = 0; i < 15; ++i) {
            mc_function f = base;
            f.params[MC_PARAM_V0] = 1.0 + (double)(i % 5) * 0.5;
            f.params[0] = 0.5 + (double)(i / 5) * 0.25;
            f.seed = base.seed + i;
            gt.push_back(f);
        }
        if (!check_results(gt, gr, false, "resident grid")) return false;
        mc_stats st;
        CHECK(mc_get_stats(ctx, &st) == MC_OK && st.bad_records == 0, "stats");
        CHECK(st.promoted == 6 + 5, "promoted %llu", (unsigned long long)st.promoted);
        CHECK(st.functions == 40 + 3 + 60 + 25 + 15 + 11, "functions %llu", (unsigned long long)st.functions);
        uint64_t pr = 1, pt = 1;
        CHECK(mc_pending(ctx, &pr, &pt) == MC_OK && pr == 0 && pt == 0, "pending");
        // a blocking request afterwards, and one on a launch context at the same time
        mc_ctx* other = create(0, 7);
        CHECK(other, "create launch context");
        if (!run_request(ctx, mixed_table(9, 104, 3), false, "resident blocking")) return false;
        if (!run_request(other, mixed_table(9, 104, 3), false, "launch context")) return false;
        mc_destroy(other);
        uint32_t fam = 0;
        // (the emulation has no run-time compiler: registration reaches it and fails there)
        CHECK(mc_register_family(ctx, "x", &fam) == MC_ERR_COMPILE, "run-time family: %s", mc_last_error(ctx));
        CHECK(mc_autotune(ctx, MC_PREC_FP32_EVAL, nullptr, 0.1) == MC_ERR_INVALID_ARG, "autotune refused");
        mc_destroy(ctx);
    }
    return true;
}

// The kernel leaves by itself after a while without work; the next request
// starts a new launch.  A context destroyed while its kernel runs stops it.
bool resident_relaunch()
{
    mc_ctx* ctx = create(MC_RESIDENT);
    CHECK(ctx, "create");
    if (!run_request(ctx, mixed_table(10, 110), false, "first")) return false;
    mc_stats st;
    CHECK(mc_get_stats(ctx, &st) == MC_OK && st.launches == 1, "launches %llu", (unsigned long long)st.launches);
    usleep(300000);  // longer than the (emulated) idle bound
    if (!run_request(ctx, mixed_table(10, 111, 4), false, "second")) return false;
    CHECK(mc_get_stats(ctx, &st) == MC_OK && st.launches == 2, "launches %llu", (unsigned long long)st.launches);
    uint64_t id = 0;
    const std::vector<mc_function> t = mixed_table(30, 112);
    CHECK(mc_submit(ctx, t.data(), t.size(), MC_PREC_FP32_EVAL, &id) == MC_OK, "submit");
    CHECK(mc_run(ctx, nullptr) == MC_OK, "run");
    mc_destroy(ctx);  // with the kernel running and the request unfinished
    return true;
}

// More runs than the record arena holds within one launch: the host ends the
// launch (the workgroups finish what they read) and starts the next, and every
// result is as expected.  Small rings of unread entries, every policy.
bool resident_flush()
{
    for (uint32_t policy : {MC_SCHED_FAIR, MC_SCHED_SRPT}) {
        mc_ctx* ctx = create(MC_RESIDENT, 3, policy, 1000, 1 << 16);  // an arena of 8192
        CHECK(ctx, "create");
        std::vector<std::vector<mc_function>> reqs;
        std::vector<uint64_t> ids;
        for (int k = 0; k < 10; ++k) {
            std::vector<mc_function> t;
            for (int i = 0; i < 1000; ++i) {
                const uint64_t seed = (200ull + k) << 32 | (uint64_t)i | (i % 97 == 1 ? 1ull << 63 : 0ull);
                t.push_back(make_fn((uint32_t)(i % 4), 1 + (uint32_t)(i % 5), i % 13 == 0 ? 20001 : 7, seed));
            }
            reqs.push_back(t);
        }
        std::vector<uint64_t> order;
        size_t submitted = 0;
        for (int guard = 0; guard < 4000000 && order.size() < reqs.size(); ++guard) {
            if (submitted < reqs.size()) {
                uint64_t id = 0;
                const mc_status st = mc_submit(ctx, reqs[submitted].data(), reqs[submitted].size(), MC_PREC_FP32_EVAL, &id);
                CHECK(st == MC_OK, "submit: %s", mc_last_error(ctx));
                ids.push_back(id);
                ++submitted;
            }
            CHECK(mc_run(ctx, nullptr) == MC_OK, "run: %s", mc_last_error(ctx));
            uint64_t got[16];
            size_t n = 0;
            CHECK(mc_poll(ctx, got, 16, &n) == MC_OK, "poll");
            for (size_t i = 0; i < n; ++i) order.push_back(got[i]);
        }
        CHECK(order.size() == reqs.size(), "requests did not all complete");
        for (size_t k = 0; k < reqs.size(); ++k) {
            std::vector<mc_result> r(reqs[k].size());
            CHECK(mc_results(ctx, ids[k], r.data(), r.size(), 0) == MC_OK, "results");
            if (!check_results(reqs[k], r, false, "flush")) return false;
        }
        mc_stats st;
        CHECK(mc_get_stats(ctx, &st) == MC_OK && st.bad_records == 0, "stats");
        CHECK(st.launches >= 2, "launches %llu", (unsigned long long)st.launches);
        std::printf("resident flush (policy %u): %llu launches, %llu functions, %llu promoted\n", policy,
                    (unsigned long long)st.launches, (unsigned long long)st.functions,
                    (unsigned long long)st.promoted);
        mc_destroy(ctx);
    }
    return true;
}

// Abort while the ring holds work: results that were in complete normally, the
// rest come back aborted; a request submitted after the call, and the next
// ones, are served normally.
bool resident_abort()
{
    mc_ctx* ctx = create(MC_RESIDENT, 2);
    CHECK(ctx, "create");
    const std::vector<mc_function> t = mixed_table(40, 120);
    uint64_t id = 0, id2 = 0;
    CHECK(mc_submit(ctx, t.data(), t.size(), MC_PREC_FP32_EVAL, &id) == MC_OK, "submit");
    CHECK(mc_submit(ctx, t.data(), 5, MC_PREC_FP64, &id2) == MC_OK, "submit");
    CHECK(mc_run(ctx, nullptr) == MC_OK, "run");
    CHECK(mc_abort(ctx) == MC_OK, "abort");
    uint64_t later = 0;
    const std::vector<mc_function> t3 = mixed_table(7, 123);
    CHECK(mc_submit(ctx, t3.data(), t3.size(), MC_PREC_FP32_EVAL, &later) == MC_OK, "submit after the abort");
    std::vector<mc_result> r(t.size());
    const mc_status st = mc_results(ctx, id, r.data(), r.size(), 1);
    CHECK(st == MC_ERR_ABORTED, "aborted request: %d", (int)st);
    if (!check_cancelled(t, r, "aborted")) return false;
    std::vector<mc_result> r2(5);
    CHECK(mc_results(ctx, id2, r2.data(), 5, 1) == MC_ERR_ABORTED, "second request aborted");
    std::vector<mc_result> r3(t3.size());
    CHECK(mc_results(ctx, later, r3.data(), r3.size(), 1) == MC_OK, "submitted after the abort: %s", mc_last_error(ctx));
    if (!check_results(t3, r3, false, "submitted after the abort")) return false;
    if (!run_request(ctx, mixed_table(12, 121, 3), false, "after abort")) return false;
    if (!run_request(ctx, mixed_table(12, 122), true, "after abort fp64")) return false;
    mc_destroy(ctx);
    return true;
}

// Checkpoint and resume: requests snapshotted part way through (functions
// spanning launches or a resident launch's chunks, promotions pending, a grid,
// one still queued, one finished), in launch and resident contexts, and
// restored into a launch and a resident context, complete with exactly the
// expected results; a request restored a moment ago snapshots to the bytes it
// came from (queued, admitted with its partials not yet copied, or copied);
// sizes, truncated and altered snapshots.
std::vector<uint8_t> take_snapshot(mc_ctx* c, uint64_t id)
{
    size_t need = 0, got = 0;
    if (mc_snapshot(c, id, nullptr, 0, &need) != MC_OK || need == 0) return {};
    std::vector<uint8_t> b(need);
    if (mc_snapshot(c, id, b.data(), b.size(), &got) != MC_OK || got != need) return {};
    return b;
}

// Two snapshots of one request state: equal but for the request id in the header.
bool same_snapshot(const std::vector<uint8_t>& x, const std::vector<uint8_t>& y)
{
    constexpr size_t kIdAt = 56, kHeader = 64;
    return x.size() == y.size() && x.size() > kHeader && std::memcmp(x.data(), y.data(), kIdAt) == 0 &&
           std::memcmp(x.data() + kHeader, y.data() + kHeader, x.size() - kHeader) == 0;
}

// Functions of a snapshot that had run part of their tiles.
uint64_t partly_run(const std::vector<uint8_t>& b, size_t n, bool grid)
{
    const size_t at = 64 + (grid ? sizeof(zmc::GridSpec) : 0) + n * sizeof(mc_function);
    uint64_t k = 0;
    for (size_t i = 0; i < n; ++i) {
        uint32_t w[4];
        std::memcpy(w, b.data() + at + 16 * i, sizeof w);
        k += w[2] > 0 && w[2] < w[1];
    }
    return k;
}

bool snapshot_restore()
{
    uint64_t partial_fns = 0;
    for (uint32_t flags : {(uint32_t)MC_NO_GRAPH, 0u, (uint32_t)MC_RESIDENT}) {
        mc_ctx* a = create(flags, 5, MC_SCHED_FAIR, 64, 1 << 14);
        CHECK(a, "create");
        // a request that has finished (results not yet taken) when it is snapshotted
        std::vector<mc_function> small = mixed_table(3, 143);
        uint64_t sid = 0;
        CHECK(mc_submit(a, small.data(), small.size(), MC_PREC_FP32_EVAL, &sid) == MC_OK, "submit small");
        bool small_done = false;
        for (int i = 0; i < 20000 && !small_done; ++i) {
            size_t n = 0;
            uint64_t got[8];
            CHECK(mc_run(a, nullptr) != MC_ERR_HIP && mc_poll(a, got, 8, &n) == MC_OK, "run");
            for (size_t k = 0; k < n; ++k) small_done = small_done || got[k] == sid;
        }
        CHECK(small_done, "small request");
        std::vector<std::vector<mc_function>> reqs = {mixed_table(20, 140, 4), mixed_table(6, 141), mixed_table(40, 142)};
        std::vector<bool> is_grid = {false, false, false};
        std::vector<uint64_t> ids;
        for (size_t k = 0; k < reqs.size(); ++k) {
            uint64_t id = 0;
            const mc_status st = mc_submit(a, reqs[k].data(), reqs[k].size(), k == 1 ? MC_PREC_FP64 : MC_PREC_FP32_EVAL, &id);
            CHECK(st == MC_OK, "submit %zu: %s", k, mc_last_error(a));
            ids.push_back(id);
        }
        const mc_function base = make_fn(MC_FAMILY_HARMONIC, 3, 50001, 7ull << 32, 1.5);
        mc_grid_axis axes[2] = {{MC_PARAM_V0, 5, 1.0, 0.5}, {0, 3, 0.5, 0.25}};
        uint64_t gid = 0;
        CHECK(mc_submit_grid(a, &base, axes, 2, MC_PREC_FP32_EVAL, &gid) == MC_OK, "grid");
        std::vector<mc_function> gt;
        for (uint64_t i = 0; i < 15; ++i) {
            mc_function f = base;
            f.params[MC_PARAM_V0] = 1.0 + (double)(i % 5) * 0.5;
            f.params[0] = 0.5 + (double)(i / 5) * 0.25;
            f.seed = base.seed + i;
            gt.push_back(f);
        }
        ids.push_back(gid);
        reqs.push_back(gt);
        is_grid.push_back(true);
        // a grid whose rows the FP32 check sends to FP64 (constant in the emulated FP32 kernel)
        const mc_function pbase = make_fn(MC_FAMILY_GAUSSIAN, 2, 30001, (1ull << 63) | (145ull << 32));
        mc_grid_axis paxis = {0, 4, 0.5, 0.25};
        uint64_t pid = 0;
        CHECK(mc_submit_grid(a, &pbase, &paxis, 1, MC_PREC_FP32_EVAL, &pid) == MC_OK, "promoted grid");
        std::vector<mc_function> pt;
        for (uint64_t i = 0; i < 4; ++i) {
            mc_function f = pbase;
            f.params[0] = 0.5 + (double)i * 0.25;
            f.seed = pbase.seed + i;
            pt.push_back(f);
        }
        ids.push_back(pid);
        reqs.push_back(pt);
        is_grid.push_back(true);
        for (int i = 0; i < 40; ++i) CHECK(mc_run(a, nullptr) != MC_ERR_HIP, "run");
        ids.push_back(sid);
        reqs.push_back(small);
        is_grid.push_back(false);
        std::vector<std::vector<uint8_t>> blobs;
        for (size_t k = 0; k < ids.size(); ++k) {
            size_t need = 0;
            CHECK(mc_snapshot(a, ids[k], nullptr, 0, &need) == MC_OK && need > 0, "size %zu: %s", k, mc_last_error(a));
            std::vector<uint8_t> b(need);
            size_t got = 0;
            const mc_status small_st = mc_snapshot(a, ids[k], b.data(), need - 1, &got);
            CHECK(small_st == MC_ERR_INVALID_ARG && got == need, "small buffer %zu (flags %u): status %d, %zu of %zu: %s", k,
                  flags, (int)small_st, got, need, mc_last_error(a));
            CHECK(mc_snapshot(a, ids[k], b.data(), b.size(), &got) == MC_OK && got == need, "snapshot %zu: %s", k,
                  mc_last_error(a));
            partial_fns += partly_run(b, reqs[k].size(), is_grid[k]);
            blobs.push_back(b);
            // the request goes on where it was (a resident launch between snapshots)
            for (int i = 0; i < 3; ++i) CHECK(mc_run(a, nullptr) != MC_ERR_HIP, "run");
        }
        uint64_t pending_r = 0, pending_t = 0;
        CHECK(mc_pending(a, &pending_r, &pending_t) == MC_OK, "pending");
        CHECK(flags == MC_RESIDENT || pending_t > 0, "work left at the snapshot");
        // the source context finishes its requests as if nothing had happened
        for (size_t k = 0; k + 1 < ids.size(); ++k) {
            std::vector<mc_result> r(reqs[k].size());
            CHECK(mc_results(a, ids[k], r.data(), r.size(), 1) == MC_OK, "source results %zu: %s", k, mc_last_error(a));
            if (!check_results(reqs[k], r, k == 1, "after the snapshot")) return false;
        }
        mc_destroy(a);

        for (uint32_t target : {flags == MC_RESIDENT ? (uint32_t)MC_NO_GRAPH : flags, (uint32_t)MC_RESIDENT}) {
            mc_ctx* b = create(target, 7, MC_SCHED_SRPT, 128, 1 << 15);
            CHECK(b, "create");
            uint8_t seg[96];
            for (int i = 0; i < 96; ++i) seg[i] = 3;  // another tiling for new requests: restored ones keep theirs
            CHECK(mc_set_tuning(b, 0, seg) == MC_OK, "tuning");
            std::vector<uint64_t> rids;
            for (size_t k = 0; k < blobs.size(); ++k) {
                uint64_t id = 0;
                CHECK(mc_restore(b, blobs[k].data(), blobs[k].size(), &id) == MC_OK, "restore %zu: %s", k,
                      mc_last_error(b));
                // snapshotted at once: admitted, its saved partials copied or (resident) not yet
                CHECK(same_snapshot(take_snapshot(b, id), blobs[k]), "restore %zu into flags %u: snapshot differs", k,
                      target);
                rids.push_back(id);
            }
            for (size_t k = 0; k < rids.size(); ++k) {
                std::vector<mc_result> r(reqs[k].size());
                CHECK(mc_results(b, rids[k], r.data(), r.size(), 1) == MC_OK, "results %zu: %s", k, mc_last_error(b));
                if (!check_results(reqs[k], r, k == 1, "restored")) return false;
            }
            mc_destroy(b);
        }
    }
    std::printf("snapshot: %llu functions were saved part way through\n", (unsigned long long)partial_fns);
    CHECK(partial_fns > 0, "no function was saved part way through");

    // a restored request still queued (no slots free) snapshots from what it holds
    {
        mc_ctx* a = create(MC_NO_GRAPH, 5, MC_SCHED_FIFO, 64, 1 << 14);
        CHECK(a, "create");
        const std::vector<mc_function> t = mixed_table(40, 146);
        uint64_t id = 0;
        CHECK(mc_submit(a, t.data(), t.size(), MC_PREC_FP32_EVAL, &id) == MC_OK, "submit");
        for (int i = 0; i < 3; ++i) CHECK(mc_run(a, nullptr) != MC_ERR_HIP, "run");
        const std::vector<uint8_t> blob = take_snapshot(a, id);
        CHECK(!blob.empty() && partly_run(blob, t.size(), false) > 0, "a snapshot part way through");
        uint64_t q = 0, q2 = 0;
        CHECK(mc_submit(a, t.data(), t.size(), MC_PREC_FP32_EVAL, &q2) == MC_OK, "submit");  // takes the free slots
        CHECK(mc_restore(a, blob.data(), blob.size(), &q) == MC_OK, "restore: %s", mc_last_error(a));
        uint64_t pr = 0, pt = 0;
        CHECK(mc_pending(a, &pr, &pt) == MC_OK && pr == 3, "three requests in the context");
        CHECK(same_snapshot(take_snapshot(a, q), blob), "queued restored request: snapshot differs");
        for (uint64_t r_id : {id, q2, q}) {
            std::vector<mc_result> r(t.size());
            CHECK(mc_results(a, r_id, r.data(), r.size(), 1) == MC_OK, "results: %s", mc_last_error(a));
            if (!check_results(t, r, false, "queued restore")) return false;
        }
        mc_destroy(a);
    }

    // damaged snapshots
    {
        const std::vector<mc_function> t = mixed_table(20, 147);
        mc_ctx* a = create(MC_NO_GRAPH, 5, MC_SCHED_FIFO, 64, 1 << 14);
        CHECK(a, "create");
        uint64_t id = 0;
        CHECK(mc_submit(a, t.data(), t.size(), MC_PREC_FP32_EVAL, &id) == MC_OK, "submit");
        for (int i = 0; i < 3; ++i) CHECK(mc_run(a, nullptr) != MC_ERR_HIP, "run");
        const std::vector<uint8_t> blob = take_snapshot(a, id);
        CHECK(!blob.empty(), "snapshot");
        std::vector<mc_result> res(t.size());
        CHECK(mc_results(a, id, res.data(), res.size(), 1) == MC_OK, "results");
        std::vector<uint8_t> bad = blob;
        bad[0] = 'X';
        CHECK(mc_restore(a, bad.data(), bad.size(), &id) == MC_ERR_INVALID_ARG, "magic");
        CHECK(mc_restore(a, blob.data(), blob.size() - 16, &id) == MC_ERR_INVALID_ARG, "truncated");
        bad = blob;
        const size_t fn_off = 64 + t.size() * sizeof(mc_function);
        bad[fn_off + 4] ^= 1;  // function 0's tile count
        CHECK(mc_restore(a, bad.data(), bad.size(), &id) == MC_ERR_INVALID_ARG, "tile count: %s", mc_last_error(a));
        mc_destroy(a);
    }
    return true;
}

// Cancellation of single requests, in every engine: a queued request completes
// at once, one whose work is running completes once nothing refers to it
// (results already in stay, the rest come back aborted), a complete one keeps
// its results; the other requests, and a request that reuses the cancelled
// one's slots, come back exactly right.
bool cancel_requests()
{
    for (uint32_t flags : {(uint32_t)MC_NO_GRAPH, 0u, (uint32_t)MC_RESIDENT}) {
        mc_ctx* ctx = create(flags, 6, MC_SCHED_FIFO, 64, 1 << 14);
        CHECK(ctx, "create");
        const std::vector<mc_function> a = mixed_table(20, 150), b = mixed_table(30, 151, 4), c = mixed_table(40, 152);
        uint64_t ia = 0, ib = 0, ic = 0;
        // b first: FIFO runs its work first, so it is on the GPU when it is cancelled
        CHECK(mc_submit(ctx, b.data(), b.size(), MC_PREC_FP32_EVAL, &ib) == MC_OK, "submit b");
        CHECK(mc_submit(ctx, a.data(), a.size(), MC_PREC_FP32_EVAL, &ia) == MC_OK, "submit a");
        CHECK(mc_submit(ctx, c.data(), c.size(), MC_PREC_FP32_EVAL, &ic) == MC_OK, "submit c");  // queued: no slots
        for (int i = 0; i < 3; ++i) CHECK(mc_run(ctx, nullptr) != MC_ERR_HIP, "run");
        // (the last launch is still in flight: no call has collected it)
        CHECK(mc_cancel(ctx, ic) == MC_OK, "cancel queued: %s", mc_last_error(ctx));
        CHECK(mc_cancel(ctx, ib) == MC_OK, "cancel running: %s", mc_last_error(ctx));
        CHECK(mc_cancel(ctx, ib) == MC_OK, "cancel twice");
        uint64_t got[16];
        size_t n = 0;
        CHECK(mc_poll(ctx, got, 16, &n) == MC_OK, "poll");
        bool seen_b = false, seen_c = false;
        for (size_t k = 0; k < n; ++k) {
            seen_b = seen_b || got[k] == ib;
            seen_c = seen_c || got[k] == ic;
        }
        CHECK(seen_c && seen_b, "cancelled requests complete once their launches are collected (flags %u)", flags);
        std::vector<mc_result> rc(c.size());
        CHECK(mc_results(ctx, ic, rc.data(), rc.size(), 0) == MC_ERR_ABORTED, "queued: aborted");
        for (const mc_result& x : rc) CHECK(x.status == MC_ERR_ABORTED, "queued: status %d", x.status);
        size_t need = 0;
        std::vector<mc_result> rb(b.size());
        CHECK(mc_results(ctx, ib, rb.data(), rb.size(), 0) == MC_ERR_ABORTED, "running: aborted (flags %u)", flags);
        if (!check_cancelled(b, rb, "running")) return false;
        CHECK(mc_snapshot(ctx, ib, nullptr, 0, &need) == MC_ERR_UNKNOWN_REQUEST, "taken");
        // a request in the cancelled one's slots
        const std::vector<mc_function> d = mixed_table(40, 153, 5);
        uint64_t id = 0;
        CHECK(mc_submit(ctx, d.data(), d.size(), MC_PREC_FP32_EVAL, &id) == MC_OK, "submit d");
        std::vector<mc_result> rd(d.size()), ra(a.size());
        CHECK(mc_results(ctx, id, rd.data(), rd.size(), 1) == MC_OK, "d: %s", mc_last_error(ctx));
        if (!check_results(d, rd, false, "after a cancel")) return false;
        // a complete request keeps its results
        for (int i = 0; i < 20000; ++i) {
            CHECK(mc_run(ctx, nullptr) != MC_ERR_HIP && mc_poll(ctx, got, 16, &n) == MC_OK, "run");
            bool a_done = false;
            for (size_t k = 0; k < n; ++k) a_done = a_done || got[k] == ia;
            if (a_done) break;
        }
        CHECK(mc_cancel(ctx, ia) == MC_OK, "cancel complete");
        CHECK(mc_results(ctx, ia, ra.data(), ra.size(), 1) == MC_OK, "a: %s", mc_last_error(ctx));
        if (!check_results(a, ra, false, "beside the cancels")) return false;
        CHECK(mc_cancel(ctx, ia) == MC_ERR_UNKNOWN_REQUEST, "unknown id");
        mc_destroy(ctx);
    }
    return true;
}

// Snapshots, restores, cancels and the odd abort interleaved with running work
// in a launch and a resident context (the emulated resident kernel runs in worker threads,
// so the interleavings vary from run to run), by seeded scripts: every request
// and every restored copy comes back exact, every cancelled one with exactly
// the results that were in.  Run under the address sanitizer, a request used
// after it was released would stop the run.
bool interleave_one(uint32_t seed, bool resident_first, int fault_at = 0, bool* saw_failure = nullptr)
{
    // with fault_at > 0, the fault_at-th checked HIP call from the first
    // context's creation on fails (either context's): a call that reports it
    // is let through, and every request must still come back exact, aborted
    // with exactly what was in, or with an error
    bool failed = false;
    auto hip_err = [&](mc_status st) {
        const bool e = fault_at > 0 && (st == MC_ERR_HIP || st == MC_ERR_OUT_OF_MEMORY);
        failed = failed || e;
        return e;
    };
    std::vector<std::vector<mc_function>> jobs;
    std::vector<bool> fp64;
    for (uint32_t k = 0; k < 8; ++k) {
        jobs.push_back(mixed_table(4 + (k * 7 + seed) % 23, 300 + seed * 16 + k, k % 3 == 1 ? 4 : 0));
        fp64.push_back(k % 4 == 3);
    }
    uint64_t state = 0x9E3779B97F4A7C15ull ^ (uint64_t)seed * 0xBF58476D1CE4E5B9ull;
    auto next = [&state](uint32_t n) {
        state ^= state << 13;
        state ^= state >> 7;
        state ^= state << 17;
        return (uint32_t)(state % n);
    };
    // (the launch context replays graphs in odd seeds; the policies rotate)
    const uint32_t launch_flags = seed % 2 ? 0u : (uint32_t)MC_NO_GRAPH;
    const uint32_t policies[3] = {MC_SCHED_FAIR, MC_SCHED_SRPT, MC_SCHED_FIFO};
    mc_ctx* b = create(resident_first ? launch_flags : MC_RESIDENT, 9, policies[(seed + 1) % 3], 128, 1 << 15);
    if (fault_at > 0) {
        char buf[32];
        std::snprintf(buf, sizeof buf, "%d", fault_at);
        setenv("MC_FAULT_HIP", buf, 1);
    }
    mc_ctx* a = create(resident_first ? MC_RESIDENT : launch_flags, 5, policies[seed % 3], 128, 1 << 15);
    unsetenv("MC_FAULT_HIP");
    CHECK(a && b, "create");
    struct Live {
        mc_ctx* ctx;
        uint64_t id;
        uint32_t job;
        bool cancelled;
        std::string how;
    };
    std::vector<Live> live;
    std::vector<uint32_t> order;
    for (uint32_t k = 0; k < jobs.size(); ++k) order.push_back(k);
    auto check = [&](const Live& l, int blocking) -> int {
        std::vector<mc_result> r(jobs[l.job].size());
        const mc_status st = mc_results(l.ctx, l.id, r.data(), r.size(), blocking);
        if (st == MC_NOT_READY) return 0;
        if (hip_err(st)) return 1;
        if (l.cancelled) {
            CHECK(st == MC_OK || st == MC_ERR_ABORTED, "seed %u: cancelled job %u: status %d", seed, l.job, (int)st);
            if (!check_cancelled(jobs[l.job], r, "interleave (cancelled)", fp64[l.job])) return -1;
        } else {
            CHECK(st == MC_OK, "seed %u: job %u: status %d: %s", seed, l.job, (int)st, mc_last_error(l.ctx));
            if (!check_results(jobs[l.job], r, fp64[l.job], "interleave")) {
                std::fprintf(stderr, "request %llu in the %s context, job %u: %s\n", (unsigned long long)l.id,
                             (l.ctx == a) == resident_first ? "resident" : "launch", l.job, l.how.c_str());
                return -1;
            }
        }
        return 1;
    };
    const bool trace = std::getenv("EMU_TRACE") != nullptr;
    for (int step = 0; step < 120; ++step) {
        const uint32_t op = next(7);
        if (trace) {
            std::fprintf(stderr, "seed %u %s step %d op %u live %zu\n", seed, resident_first ? "res" : "launch", step, op,
                         live.size());
            std::fflush(stderr);
        }
        if (op == 0 && !order.empty()) {
            const uint32_t k = order[next((uint32_t)order.size())];
            order.erase(std::find(order.begin(), order.end(), k));
            uint64_t id = 0;
            const mc_status ss =
                mc_submit(a, jobs[k].data(), jobs[k].size(), fp64[k] ? MC_PREC_FP64 : MC_PREC_FP32_EVAL, &id);
            if (hip_err(ss)) continue;
            CHECK(ss == MC_OK, "submit: %s", mc_last_error(a));
            live.push_back(Live{a, id, k, false, "submitted at step " + std::to_string(step)});
        } else if (op == 1) {
            std::vector<size_t> cand;
            for (size_t i = 0; i < live.size(); ++i)
                if (!live[i].cancelled) cand.push_back(i);
            if (cand.empty()) continue;
            const Live src = live[cand[next((uint32_t)cand.size())]];
            const std::vector<uint8_t> blob = take_snapshot(src.ctx, src.id);
            mc_ctx* dst = next(2) ? a : b;
            if (blob.empty() && fault_at > 0) {  // (a HIP failure, or a request lost to one)
                failed = true;
                continue;
            }
            CHECK(!blob.empty(), "seed %u: snapshot: %s", seed, mc_last_error(src.ctx));
            uint64_t id = 0;
            const mc_status rs = mc_restore(dst, blob.data(), blob.size(), &id);
            if (hip_err(rs)) continue;
            CHECK(rs == MC_OK, "restore: %s", mc_last_error(dst));
            live.push_back(Live{dst, id, src.job, false,
                                "restored at step " + std::to_string(step) + " from request " + std::to_string(src.id) +
                                    " (" + src.how + ")"});
        } else if (op == 2) {
            const mc_status ra = mc_run(a, nullptr), rb = mc_run(b, nullptr);
            CHECK((ra != MC_ERR_HIP || hip_err(ra)) && (rb != MC_ERR_HIP || hip_err(rb)), "run");
        } else if (op == 3) {
            for (mc_ctx* c : {a, b}) {
                uint64_t got[64];
                size_t n = 0;
                const mc_status ps = mc_poll(c, got, 64, &n);
                if (hip_err(ps)) continue;
                CHECK(ps == MC_OK, "poll");
                for (size_t j = 0; j < n; ++j) {
                    auto it = std::find_if(live.begin(), live.end(),
                                           [&](const Live& l) { return l.ctx == c && l.id == got[j]; });
                    CHECK(it != live.end(), "seed %u: polled id %llu unknown", seed, (unsigned long long)got[j]);
                    const int rc = check(*it, 0);
                    CHECK(rc == 1, "seed %u: a polled request is not ready (%d)", seed, rc);
                    live.erase(it);
                }
            }
        } else if (op == 5) {
            std::vector<size_t> cand;
            for (size_t i = 0; i < live.size(); ++i)
                if (!live[i].cancelled) cand.push_back(i);
            if (cand.size() <= 2) continue;
            Live& l = live[cand[next((uint32_t)cand.size())]];
            const mc_status cs = mc_cancel(l.ctx, l.id);
            CHECK(cs == MC_OK || hip_err(cs), "seed %u: cancel: %s", seed, mc_last_error(l.ctx));
            l.cancelled = true;
        } else if (op == 4 && next(8) == 0) {
            // abort one context: every request in it so far keeps what came in
            mc_ctx* c = next(2) ? a : b;
            const mc_status as = mc_abort(c);
            CHECK(as == MC_OK || hip_err(as), "seed %u: abort", seed);
            for (Live& l : live)
                if (l.ctx == c) l.cancelled = true;
        } else {
            const mc_status ra = mc_run(a, nullptr);
            CHECK(ra != MC_ERR_HIP || hip_err(ra), "run");
        }
    }
    for (const Live& l : live) {
        if (trace) {
            std::fprintf(stderr, "end: waiting for request %llu in the %s context, job %u, %s%s\n",
                         (unsigned long long)l.id, (l.ctx == a) == resident_first ? "resident" : "launch", l.job,
                         l.how.c_str(), l.cancelled ? ", cancelled" : "");
            std::fflush(stderr);
        }
        CHECK(check(l, 1) == 1, "seed %u: results at the end", seed);
    }
    mc_destroy(a);
    mc_destroy(b);
    if (saw_failure) *saw_failure = failed;
    return true;
}

bool interleave()
{
    for (uint32_t seed = 1; seed <= 24; ++seed)
        for (bool resident_first : {false, true})
            if (!interleave_one(seed, resident_first)) {
                std::fprintf(stderr, "interleave: seed %u, %s first\n", seed, resident_first ? "resident" : "launch");
                return false;
            }
    return true;
}

// The same scripts with one checked HIP call failing in each run, at points
// spread over the scripts' calls.
bool interleave_faults()
{
    int runs = 0, saw = 0;
    for (int base : {3, 40, 111})
        for (uint32_t seed = 1; seed <= 24; ++seed)
            for (bool resident_first : {false, true}) {
                const int at = base + (int)seed * 53;
                bool failed = false;
                if (!interleave_one(seed, resident_first, at, &failed)) {
                    std::fprintf(stderr, "interleave_faults: seed %u, %s first, failing call %d\n", seed,
                                 resident_first ? "resident" : "launch", at);
                    return false;
                }
                ++runs;
                saw += failed ? 1 : 0;
            }
    CHECK(saw > runs / 5, "only %d of %d runs saw the failure", saw, runs);
    std::printf("interleave_faults: %d runs, %d of them saw a failed HIP call\n", runs, saw);
    return true;
}

// The packing's own hypot and atan2 (built from correctly rounded operations so
// that host and device pack the same bits) against libm: within a few units in
// the last place, over magnitudes 10^-6..10^6, zeros, equal and opposite values.
bool pack_math()
{
    uint64_t s = 0x9E3779B97F4A7C15ull;
    auto next = [&s]() {
        s ^= s << 13;
        s ^= s >> 7;
        s ^= s << 17;
        return (double)(s >> 11) * 0x1p-53 * 2.0 - 1.0;
    };
    double worst_h = 0.0, worst_a = 0.0;
    for (int i = 0; i < 400000; ++i) {
        double a = next() * std::pow(10.0, 6.0 * next()), b = next() * std::pow(10.0, 6.0 * next());
        if (i % 7 == 0) b = 0.0;
        if (i % 11 == 0) a = 0.0;
        if (i % 13 == 0) b = a;
        if (i % 17 == 0) b = -a;
        const double h = std::hypot(a, b);
        worst_h = std::max(worst_h, std::fabs(zmc::pack_hypot(a, b) - h) / (h > 0.0 ? h : 1.0));
        double e = std::fabs(zmc::pack_atan2(b, a) - ((a == 0.0 && b == 0.0) ? 0.0 : std::atan2(b, a)));
        if (std::fabs(e - 2.0 * M_PI) < 1e-9) e = std::fabs(e - 2.0 * M_PI);  // the angle of -0 may land on -pi or pi
        worst_a = std::max(worst_a, e);
    }
    CHECK(worst_h <= 4.5e-16, "pack_hypot: relative error %.3g", worst_h);
    CHECK(worst_a <= 8.9e-16, "pack_atan2: error %.3g rad", worst_a);
    std::printf("pack_hypot within %.2g relative, pack_atan2 within %.2g rad of libm\n", worst_h, worst_a);
    return true;
}

// MC_LOG=3: the context, its launches and admissions, the resident kernel's
// launch and exit, and a failure each leave a "[zmc] " line on stderr; MC_LOG
// unset leaves none.
bool log_levels()
{
    char path[] = "/tmp/zmc_log_XXXXXX";
    const int fd = mkstemp(path);
    CHECK(fd >= 0, "mkstemp");
    std::fflush(stderr);
    const int saved = dup(2);
    dup2(fd, 2);
    bool ok = true;
    for (int level : {0, 3}) {
        if (level) setenv("MC_LOG", "3", 1);
        else unsetenv("MC_LOG");
        mc_ctx* a = create(0, 7);
        mc_ctx* b = create(MC_RESIDENT);
        ok = ok && a && b;
        if (ok) {
            ok = run_request(a, mixed_table(6, 130, 3), false, "log launch") &&
                 run_request(b, mixed_table(6, 131), false, "log resident");
            uint64_t id = 0;
            std::vector<mc_function> bad = mixed_table(3, 132);
            bad[1].dim = 0;
            ok = ok && mc_submit(a, bad.data(), bad.size(), MC_PREC_FP32_EVAL, &id) == MC_ERR_BAD_DIM;
        }
        if (a) mc_destroy(a);
        if (b) mc_destroy(b);
        std::fflush(stderr);
        if (level == 0) {
            ok = ok && lseek(fd, 0, SEEK_END) == 0;  // nothing written
        }
    }
    unsetenv("MC_LOG");
    std::fflush(stderr);
    dup2(saved, 2);
    close(saved);
    std::string text;
    {
        FILE* f = std::fopen(path, "r");
        char buf[4096];
        size_t n;
        while (f && (n = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, n);
        if (f) std::fclose(f);
    }
    close(fd);
    std::remove(path);
    CHECK(ok, "runs with logging: %s", text.c_str());
    for (const char* want : {"[zmc] context on device 0", "[zmc] launch 1: ", "admitted: 6 functions",
                             "[zmc] resident launch 1: ", "[zmc] error -3: function 1:", "resident"})
        CHECK(text.find(want) != std::string::npos, "no line with \"%s\" in:\n%s", want, text.c_str());
    return true;
}

}  // namespace

int main(int argc, char** argv)
{
    const std::map<std::string, bool (*)()> all = {
        {"basic", basic},     {"many_launches", many_launches}, {"admission", admission},
        {"grid", grid},       {"abort", abort_and_continue},    {"errors", errors},
        {"plain", plain_paths}, {"two_contexts", two_contexts}, {"fault_sweep", fault_sweep},
        {"autotune_cache", autotune_cache}, {"resident_basic", resident_basic},
        {"resident_relaunch", resident_relaunch}, {"resident_flush", resident_flush},
        {"resident_abort", resident_abort}, {"log_levels", log_levels}, {"snapshot", snapshot_restore},
        {"pack_math", pack_math}, {"cancel", cancel_requests}, {"interleave", interleave},
        {"interleave_faults", interleave_faults},
    };
    std::vector<std::string> names;
    for (int i = 1; i < argc; ++i) {
        if (std::string(argv[i]) == "all")
            for (const auto& kv : all) names.push_back(kv.first);
        else
            names.push_back(argv[i]);
    }
    for (const std::string& s : names) {
        auto it = all.find(s);
        if (it == all.end()) {
            std::fprintf(stderr, "unknown scenario %s\n", s.c_str());
            return 2;
        }
        if (!it->second()) {
            std::fprintf(stderr, "FAILED %s\n", s.c_str());
            return 1;
        }
        std::printf("ok %s\n", s.c_str());
        std::fflush(stdout);
    }
    return g_failures == 0 ? 0 : 1;
}
