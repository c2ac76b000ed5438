/*
 * A plain C client of libzmc (include/zmc.h), for the tests: reads an array of
 * mc_function records from a file, integrates them through the C ABI alone --
 * the batched path in FP32 evaluation and in FP64 (submitted together, launched
 * with mc_run, collected with mc_poll and mc_results), the plain FP64 path, and
 * FP32 evaluation through a resident context (MC_RESIDENT) -- and writes the
 * four mc_result arrays, one after another, to the output file.
 * It also checks that an invalid function is rejected with MC_ERR_BAD_DIM and a
 * message.  Usage: zmc_c_client <functions.bin> <results.bin>.  Exit status 0 on
 * success; on failure the status and mc_last_error go to stderr.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#include "zmc.h"

static int check(mc_ctx* ctx, mc_status st, const char* what)
{
    if (st == MC_OK) return 0;
    fprintf(stderr, "%s failed: status %d: %s\n", what, (int)st, mc_last_error(ctx));
    return 1;
}

int main(int argc, char** argv)
{
    if (argc != 3) {
        fprintf(stderr, "usage: %s <functions.bin> <results.bin>\n", argv[0]);
        return 2;
    }
    FILE* in = fopen(argv[1], "rb");
    if (!in) {
        perror(argv[1]);
        return 2;
    }
    fseek(in, 0, SEEK_END);
    const long bytes = ftell(in);
    fseek(in, 0, SEEK_SET);
    if (bytes <= 0 || bytes % (long)sizeof(mc_function) != 0) {
        fprintf(stderr, "%s: %ld bytes is not a whole number of %zu-byte records\n", argv[1], bytes,
                sizeof(mc_function));
        fclose(in);
        return 2;
    }
    const size_t n = (size_t)bytes / sizeof(mc_function);
    mc_function* fns = (mc_function*)malloc((size_t)bytes);
    mc_result* res = (mc_result*)calloc(4 * n, sizeof(mc_result));
    if (!fns || !res || fread(fns, sizeof(mc_function), n, in) != n) {
        fprintf(stderr, "reading %s failed\n", argv[1]);
        fclose(in);
        return 2;
    }
    fclose(in);

    mc_config cfg;
    mc_ctx* ctx = NULL;
    int bad = check(NULL, mc_config_init(&cfg), "mc_config_init");
    cfg.flags = MC_NO_GRAPH;
    bad = bad || check(NULL, mc_create(&cfg, &ctx), "mc_create");
    if (bad) return 1;

    /* an invalid function is rejected as a whole request, with a message */
    mc_function wrong = fns[0];
    wrong.dim = MC_MAX_DIM + 1;
    uint64_t id_wrong = 0;
    const mc_status st_wrong = mc_submit(ctx, &wrong, 1, MC_PREC_FP32_EVAL, &id_wrong);
    if (st_wrong != MC_ERR_BAD_DIM || strlen(mc_last_error(ctx)) == 0) {
        fprintf(stderr, "invalid dim: expected MC_ERR_BAD_DIM with a message, got %d\n", (int)st_wrong);
        bad = 1;
    }

    uint64_t id32 = 0, id64 = 0;
    bad = bad || check(ctx, mc_submit(ctx, fns, n, MC_PREC_FP32_EVAL, &id32), "mc_submit (FP32)");
    bad = bad || check(ctx, mc_submit(ctx, fns, n, MC_PREC_FP64, &id64), "mc_submit (FP64)");
    /* launch until both requests are reported complete */
    int done32 = 0, done64 = 0;
    const time_t t0 = time(NULL);
    while (!bad && !(done32 && done64)) {
        if (time(NULL) - t0 > 60) {
            fprintf(stderr, "requests did not complete within 60 s\n");
            bad = 1;
            break;
        }
        const mc_status st = mc_run(ctx, NULL);
        if (st != MC_OK && st != MC_NOT_READY) bad = check(ctx, st, "mc_run");
        uint64_t ids[8];
        size_t got = 0;
        bad = bad || check(ctx, mc_poll(ctx, ids, 8, &got), "mc_poll");
        for (size_t i = 0; i < got; ++i) {
            if (ids[i] == id32) done32 = 1;
            if (ids[i] == id64) done64 = 1;
        }
    }
    bad = bad || check(ctx, mc_results(ctx, id32, res, n, 0), "mc_results (FP32)");
    bad = bad || check(ctx, mc_results(ctx, id64, res + n, n, 0), "mc_results (FP64)");
    bad = bad || check(ctx, mc_integrate_plain_fp64(ctx, fns, n, res + 2 * n, NULL), "mc_integrate_plain_fp64");
    mc_stats stats;
    bad = bad || check(ctx, mc_get_stats(ctx, &stats), "mc_get_stats");
    if (!bad && stats.bad_records != 0) {
        fprintf(stderr, "%llu records failed the kernels' checks\n", (unsigned long long)stats.bad_records);
        bad = 1;
    }
    bad = check(ctx, mc_destroy(ctx), "mc_destroy") || bad;
    if (bad) return 1;

    /* the same FP32 request served by a resident kernel: mc_run feeds its ring */
    mc_ctx* rctx = NULL;
    cfg.flags = MC_RESIDENT;
    bad = check(NULL, mc_create(&cfg, &rctx), "mc_create (resident)");
    uint64_t idr = 0;
    bad = bad || check(rctx, mc_submit(rctx, fns, n, MC_PREC_FP32_EVAL, &idr), "mc_submit (resident)");
    int doner = 0;
    const time_t t1 = time(NULL);
    while (!bad && !doner) {
        if (time(NULL) - t1 > 60) {
            fprintf(stderr, "the resident request did not complete within 60 s\n");
            bad = 1;
            break;
        }
        bad = check(rctx, mc_run(rctx, NULL), "mc_run (resident)");
        uint64_t ids[8];
        size_t got = 0;
        bad = bad || check(rctx, mc_poll(rctx, ids, 8, &got), "mc_poll (resident)");
        for (size_t i = 0; i < got; ++i)
            if (ids[i] == idr) doner = 1;
    }
    bad = bad || check(rctx, mc_results(rctx, idr, res + 3 * n, n, 0), "mc_results (resident)");
    if (rctx) bad = check(rctx, mc_destroy(rctx), "mc_destroy (resident)") || bad;
    if (bad) return 1;

    FILE* out = fopen(argv[2], "wb");
    if (!out || fwrite(res, sizeof(mc_result), 4 * n, out) != 4 * n) {
        perror(argv[2]);
        return 2;
    }
    fclose(out);
    printf("%zu functions: FP32, FP64, plain FP64 and resident FP32 results written (%llu launches)\n", n,
           (unsigned long long)stats.launches);
    free(fns);
    free(res);
    return 0;
}
