// Auto-tuning: the best tile configuration differs per platform and shape
// (Section 2: tile size must be tuned to the architecture), so every valid
// configuration is timed on the caller's buffers and the fastest is kept.
#include <cstdio>
#include <cstring>
#include <vector>

#include "common.h"

using namespace xc;

static std::vector<xc_config> candidates(xc_in_type in_type) {
    std::vector<xc_config> v;
    v.push_back(xc_config{XC_KERNEL_MFMA, 32, 0, 0, 0, 0});
    if (in_type != XC_IN_CF32) {   // both stagings (straight into LDS needs whole granules)
        v.push_back(xc_config{XC_KERNEL_MFMA, 64, 0, 1, XC_STAGING_LDS, 0});
        v.push_back(xc_config{XC_KERNEL_MFMA, 64, 0, 1, XC_STAGING_REGISTERS, 0});
    } else {   // one or two time groups, four or three real products
        for (int ts = 1; ts <= 2; ++ts)
            for (int pr = XC_PRODUCT_FOUR; pr <= XC_PRODUCT_THREE; ++pr)
                v.push_back(xc_config{XC_KERNEL_MFMA, 64, 0, ts, 0, pr});
        const int opts[][2] = {{16, 1}, {16, 2}, {16, 4}, {32, 2}, {32, 4}, {32, 8}};
        for (auto &o : opts) v.push_back(xc_config{XC_KERNEL_VALU, 32, o[0], o[1], 0, 0});
    }
    return v;
}

extern "C" {

xc_status xc_autotune(const void *samples, xc_in_type in_type, int32_t n_stations, int32_t n_pol,
                      int32_t n_channels, int32_t n_times, void *vis, xc_out_type out_type, const char *cache_path,
                      void *stream, xc_config *best, double *best_ms) {
    if (!best || !best_ms) return set_error(XC_ERR_INVALID_ARG, "null output pointer");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return set_error(XC_ERR_HIP, "hipEventCreate failed");
    double best_t = 1e300;
    xc_config best_c{};
    bool found = false;
    xc_status last = XC_OK;
    for (const xc_config &c : candidates(in_type)) {
        xc_config r;
        xc_status st = xc_resolve_config(&c, in_type, out_type, n_stations, n_pol, n_channels, n_times, &r);
        if (st != XC_OK) {
            last = st;
            continue;
        }
        // one warm-up, then the best of three
        st = xc_correlate_config(&r, samples, in_type, n_stations, n_pol, n_channels, n_times, vis, out_type, 0,
                                 stream);
        if (st != XC_OK) {
            last = st;
            continue;
        }
        double t_min = 1e300;
        for (int rep = 0; rep < 3 && st == XC_OK; ++rep) {
            (void)hipEventRecord(e0, s);
            st = xc_correlate_config(&r, samples, in_type, n_stations, n_pol, n_channels, n_times, vis, out_type,
                                     0, stream);
            (void)hipEventRecord(e1, s);
            if (hipEventSynchronize(e1) != hipSuccess) st = set_error(XC_ERR_HIP, "event sync failed");
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (st == XC_OK && ms < t_min) t_min = ms;
        }
        if (st != XC_OK) {
            last = st;
            continue;
        }
        if (t_min < best_t) {
            best_t = t_min;
            best_c = r;
            found = true;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!found) return last != XC_OK ? last : set_error(XC_ERR_UNSUPPORTED, "no configuration ran");
    *best = best_c;
    *best_ms = best_t;
    tune_put(TuneKey{(int)in_type, (int)out_type, n_stations, n_channels, n_times}, best_c);
    if (cache_path) {
        FILE *f = fopen(cache_path, "a");
        if (f) {
            fprintf(f,
                    "{\"in\": %d, \"out\": %d, \"S\": %d, \"C\": %d, \"T\": %d, \"kernel\": %d, \"block\": %d, "
                    "\"time_chunk\": %d, \"time_split\": %d, \"staging\": %d, \"product\": %d, \"ms\": %.6f}\n",
                    (int)in_type, (int)out_type, n_stations, n_channels, n_times, best_c.kernel, best_c.block,
                    best_c.time_chunk, best_c.time_split, best_c.staging, best_c.product, best_t);
            fclose(f);
        }
    }
    return XC_OK;
}

int64_t xc_tune_cache_load(const char *cache_path) {
    if (!cache_path) return -1;
    FILE *f = fopen(cache_path, "r");
    if (!f) return -1;
    char line[512];
    int64_t n = 0;
    while (fgets(line, sizeof line, f)) {
        int in, out, S, C, T, k, b, tc, ts, sg, pr;
        double ms;
        if (sscanf(line,
                   " {\"in\": %d, \"out\": %d, \"S\": %d, \"C\": %d, \"T\": %d, \"kernel\": %d, \"block\": %d, "
                   "\"time_chunk\": %d, \"time_split\": %d, \"staging\": %d, \"product\": %d, \"ms\": %lf",
                   &in, &out, &S, &C, &T, &k, &b, &tc, &ts, &sg, &pr, &ms) == 12) {
            xc_config c{k, b, tc, ts, sg, pr};
            xc_config r;
            if (xc_resolve_config(&c, (xc_in_type)in, (xc_out_type)out, S, 2, C, T, &r) == XC_OK) {
                tune_put(TuneKey{in, out, S, C, T}, r);
                ++n;
            }
        }
    }
    fclose(f);
    return n;
}

}  // extern "C"
