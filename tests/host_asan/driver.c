/*
 * Host-side checks of the library under AddressSanitizer (host code only; no
 * GPU is needed): every call below either is pure host logic or must reject
 * its arguments, or fail cleanly, before touching a device.  Built and run by
 * tests/test_host_asan.py; prints "ok" and exits 0 when every check holds.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "xengine.h"

static int failures = 0;
#define CHECK(cond)                                                        \
    do {                                                                   \
        if (!(cond)) {                                                     \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                                    \
        }                                                                  \
    } while (0)

int main(int argc, char **argv) {
    const char *tmpdir = argc > 1 ? argv[1] : "/tmp";

    /* status strings, version */
    for (int s = 0; s <= 12; ++s) CHECK(xc_status_string((xc_status)s) != NULL);
    CHECK(xc_version() != NULL && strlen(xc_version()) > 0);

    /* index and size helpers */
    CHECK(xc_n_baselines(1) == 1 && xc_n_baselines(64) == 2080 && xc_n_baselines(512) == 131328);
    CHECK(xc_baseline_index(0, 0) == 0 && xc_baseline_index(0, 1) == 1 && xc_baseline_index(1, 1) == 2);
    CHECK(xc_vis_elems(64, 2, 256) == (int64_t)256 * 2080 * 4);
    CHECK(xc_flops(64, 256, 768) == 32.0 * 256 * 768 * 2080);

    /* quantiles (nearest rank), including the degenerate inputs */
    double v[7] = {5, 1, 4, 2, 3, 7, 6};
    CHECK(xc_quantile(v, 7, 0.5) == 4.0 && xc_quantile(v, 7, 1.0) == 7.0 && xc_quantile(v, 7, 0.0) == 1.0);
    CHECK(v[0] == 5 && v[6] == 6);                      /* input left as it was */
    CHECK(isnan(xc_quantile(v, 0, 0.5)) && isnan(xc_quantile(NULL, 3, 0.5)));

    /* batch work lists: full, truncated, and rejected */
    const int32_t bs[3] = {24, 130, 1}, bc[3] = {5, 2, 4}, bt[3] = {768, 128, 33};
    const int64_t n = xc_batch_worklist(bs, bc, bt, 3, 64, NULL, 0, NULL);
    CHECK(n == 5 * 1 + 2 * 6 + 4 * 1);
    int32_t *units = (int32_t *)malloc(sizeof(int32_t) * 4 * (size_t)n);
    int32_t bounds[9];
    CHECK(xc_batch_worklist(bs, bc, bt, 3, 64, units, n, bounds) == n);
    CHECK(bounds[0] == 0 && bounds[8] == n);
    CHECK(xc_batch_worklist(bs, bc, bt, 3, 64, units, 2, NULL) == n);    /* writes only 2 */
    CHECK(xc_batch_worklist(bs, bc, bt, 0, 64, units, n, NULL) == 0);     /* an empty list */
    CHECK(xc_batch_worklist(bs, bc, bt, -1, 64, units, n, NULL) == -1);
    const int32_t zero_s[1] = {0};
    CHECK(xc_batch_worklist(zero_s, bc, bt, 1, 64, units, n, NULL) == -1);
    free(units);

    /* configuration resolution and tuning candidates */
    xc_config r;
    CHECK(xc_resolve_config(NULL, XC_IN_CF32, XC_OUT_CF32, 64, 2, 256, 768, &r) == XC_OK);
    xc_config bad = {XC_KERNEL_VALU, 0, 0, 3, 0, 0, 0, 0};
    CHECK(xc_resolve_config(&bad, XC_IN_CF32, XC_OUT_CF32, 64, 2, 256, 768, &r) == XC_ERR_INVALID_ARG);
    CHECK(strlen(xc_last_error()) > 0);
    xc_config cands[64];
    const int nc = xc_tune_candidates(XC_IN_CF32, cands, 64);
    CHECK(nc > 4 && nc <= 64);
    CHECK(xc_tune_candidates(XC_IN_CI8, cands, 1) >= 1);

    /* tuning cache: valid, malformed, over-long and missing files */
    char path[512];
    snprintf(path, sizeof path, "%s/tune_asan.jsonl", tmpdir);
    FILE *f = fopen(path, "w");
    CHECK(f != NULL);
    if (f) {
        fprintf(f, "{\"in\": 0, \"out\": 1, \"sb\": 2, \"gran\": 1, \"tb\": 10, \"ub\": 10, \"kernel\": 2, "
                   "\"block\": 64, \"time_chunk\": 0, \"time_split\": 2, \"staging\": 0, \"product\": 0, "
                   "\"tile_w\": 0, \"tile_h\": 0, \"ms\": 0.1, \"S\": 64, \"C\": 256, \"T\": 768}\n");
        fprintf(f, "{\"in\": 0, \"out\": 1, garbage\n");
        for (int i = 0; i < 3000; ++i) fputc('x', f);
        fputc('\n', f);
        fclose(f);
    }
    CHECK(xc_tune_cache_load(path) >= 0);
    snprintf(path, sizeof path, "%s/no_such_dir/none.jsonl", tmpdir);
    CHECK(xc_tune_cache_load(path) == -1 && xc_tune_cache_load(NULL) == -1);

    /* calls rejected before any device work */
    CHECK(xc_correlate(NULL, XC_IN_CF32, 8, 2, 1, 1, NULL, XC_OUT_CF32, 0, NULL) == XC_ERR_INVALID_ARG);
    char dummy[64];
    CHECK(xc_correlate(dummy, (xc_in_type)9, 8, 2, 1, 1, dummy, XC_OUT_CF32, 0, NULL) == XC_ERR_INVALID_ARG);
    CHECK(xc_correlate(dummy, XC_IN_CF32, 8, 3, 1, 1, dummy, XC_OUT_CF32, 0, NULL) != XC_OK);
    CHECK(xc_correlate(dummy, XC_IN_CF32, 8, 2, 1, 1, dummy, XC_OUT_CI32, 0, NULL) != XC_OK);
    CHECK(xc_correlate_split_bytes(64, 2, 256, 768, 4) > 0);

    /* streams: descriptor validation, admission against a given budget, and
       a stream whose device allocation fails cleanly without a GPU */
    xc_stream_desc d;
    memset(&d, 0, sizeof d);
    d.n_stations = 20; d.n_pol = 2; d.n_channels = 3; d.block_times = 16; d.blocks_per_integration = 4;
    d.blocks_per_fold = 2; d.ring_blocks = 4; d.in_type = XC_IN_CI8; d.acc_type = XC_OUT_CI32; d.staggered = 1;
    const size_t fp = xc_stream_footprint(&d);
    CHECK(fp > 0);
    xc_server *srv = NULL;
    CHECK(xc_server_create(fp + fp / 2, &srv) == XC_OK && srv != NULL);
    int32_t id = -1;
    xc_stream_desc bad_d = d;
    bad_d.ring_blocks = 1;
    CHECK(xc_stream_open(srv, &bad_d, &id) == XC_ERR_INVALID_ARG);
    xc_stream_desc big = d;
    big.n_channels = 3000;
    CHECK(xc_stream_open(srv, &big, &id) == XC_ERR_ADMISSION);
    const xc_status st = xc_stream_open(srv, &d, &id);
    if (st == XC_OK) CHECK(xc_stream_close(srv, id) == XC_OK);   /* a GPU is present after all */
    else CHECK(st == XC_ERR_HIP || st == XC_ERR_OUT_OF_MEMORY);
    CHECK(xc_stream_close(srv, 99) == XC_ERR_INVALID_ARG);
    bad_d = d;
    bad_d.staggered = 3;
    CHECK(xc_stream_open(srv, &bad_d, &id) == XC_ERR_INVALID_ARG);
    CHECK(xc_server_set_fold_order(srv, 1) == XC_OK && xc_server_set_fold_order(srv, 0) == XC_OK);
    CHECK(xc_server_set_fold_order(srv, 2) == XC_ERR_INVALID_ARG);
    CHECK(xc_server_set_fold_order(NULL, 1) == XC_ERR_INVALID_ARG);
    CHECK(xc_stream_flush(srv, 99) == XC_ERR_INVALID_ARG);
    xc_server_destroy(srv);

    /* the fold schedule on the host: counting, a full and a truncated listing */
    xc_stream_desc sd = d;
    sd.staggered = 2;
    int64_t nf = -1, pub[4];
    CHECK(xc_stream_schedule(&sd, 11, 1, NULL, 0, &nf, pub, 4) == XC_OK && nf > 0);
    int64_t *rows = (int64_t *)malloc((size_t)nf * 6 * sizeof(int64_t));
    int64_t nf2 = -1;
    CHECK(rows != NULL && xc_stream_schedule(&sd, 11, 1, rows, nf, &nf2, pub, 4) == XC_OK && nf2 == nf);
    CHECK(rows[4] == 0 && pub[0] >= 3 && pub[1] >= 7 && pub[2] == -1 && pub[3] == -1);
    CHECK(xc_stream_schedule(&sd, 11, 1, rows, 1, &nf2, pub, 1) == XC_OK && nf2 == nf);
    CHECK(xc_stream_schedule(&sd, 11, 3, rows, 1, &nf2, pub, 1) == XC_ERR_INVALID_ARG);
    CHECK(xc_stream_schedule(&sd, 11, 0, rows, 1, NULL, pub, 1) == XC_ERR_INVALID_ARG);
    free(rows);

    if (failures) {
        fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    printf("ok\n");
    return 0;
}
