// Auto-tuning: the best tile configuration differs per platform and shape
// (Section 2: the tile size must be tuned to the architecture), so the
// configurations of a shape are timed on the caller's buffers and the fastest
// is kept for the shape's bucket (see TuneKey).
//
// The candidates span the kernel families and their parameters: matrix-core
// blocks of 32 or 64 stations, direct-to-LDS or register staging (int8 and
// 16-bit samples), one or two time groups and three or four real products
// (complex float32 on 64-station matrix-core blocks), and for the vector-ALU
// kernel every register tile w x h (w, h in {2, 4, 8}) with every time chunk
// and time-group count.  Register tiles are pruned with Table 1 before any
// timing: a tile needs at least 4 (1 + min(w, h)) + 8 w h registers, and the
// ones that, with the kernel's staging and address registers, do not fit a
// lane's 256 are dropped (8 x 4, 4 x 8, 8 x 8); a tile and its mirror image
// cost the same on a square block pair, so only one of them is built.
#include <cstdio>
#include <cstring>
#include <vector>

#include "common.h"
#include "log.h"

using namespace xc;

namespace {

// Registers a vector-ALU lane needs beyond its Table 1 minimum: the sample
// loads in flight for the next chunk (one float4 per 16-byte element, spread
// over the workgroup) and about two dozen for addresses and loop state.
int valu_overhead_regs(int w, int h, int tc, int ts) {
    const int threads = (32 / w) * (32 / h) * ts;
    const int loads = (tc * 64 + threads - 1) / threads;
    return 4 * loads + 24;
}

std::vector<xc_config> candidates(xc_in_type in_type) {
    std::vector<xc_config> v;
    v.push_back(xc_config{XC_KERNEL_MFMA, 32, 0, 0, 0, 0, 0, 0});
    if (in_type != XC_IN_CF32) {   // both stagings
        v.push_back(xc_config{XC_KERNEL_MFMA, 64, 0, 1, XC_STAGING_LDS, 0, 0, 0});
        v.push_back(xc_config{XC_KERNEL_MFMA, 64, 0, 1, XC_STAGING_REGISTERS, 0, 0, 0});
        return v;
    }
    // arrays of at most 16 stations: one workgroup per channel (skipped for
    // larger arrays, where it does not resolve)
    v.push_back(xc_config{XC_KERNEL_VALU, 16, 0, 0, 0, 0, 0, 0});
    // one or two time groups, four or three real products
    for (int ts = 1; ts <= 2; ++ts)
        for (int pr = XC_PRODUCT_FOUR; pr <= XC_PRODUCT_THREE; ++pr)
            v.push_back(xc_config{XC_KERNEL_MFMA, 64, 0, ts, 0, pr, 0, 0});
    const int tcts[][2] = {{16, 1}, {16, 2}, {16, 4}, {32, 2}, {32, 4}, {32, 8}};
    for (int w = 2; w <= 8; w *= 2)
        for (int h = 2; h <= w; h *= 2) {       // mirror images (h > w) cost the same
            int64_t flops, bytes, regs;
            if (xc_tile_cost(w, h, &flops, &bytes, &regs) != XC_OK) continue;
            for (auto &o : tcts) {
                if (regs + valu_overhead_regs(w, h, o[0], o[1]) > 256) continue;   // Table 1 pruning
                if (!valu_available(w, h, o[0], o[1])) continue;
                v.push_back(xc_config{XC_KERNEL_VALU, 32, o[0], o[1], 0, 0, w, h});
            }
        }
    return v;
}

}  // namespace

extern "C" {

int64_t xc_tune_candidates(xc_in_type in_type, xc_config *out, int64_t capacity) {
    if (in_type < XC_IN_CF32 || in_type > XC_IN_CBF16) return -1;
    const std::vector<xc_config> v = candidates(in_type);
    for (int64_t k = 0; out && k < (int64_t)v.size() && k < capacity; ++k) out[k] = v[(size_t)k];
    return (int64_t)v.size();
}

xc_status xc_tune_bucket(xc_in_type in_type, xc_out_type out_type, int32_t n_stations, int32_t n_channels,
                         int32_t n_times, int32_t key[6]) {
    if (!key) return set_error(XC_ERR_INVALID_ARG, "null key");
    if (n_stations < 1 || n_channels < 1 || n_times < 1) return set_error(XC_ERR_INVALID_ARG, "sizes must be >= 1");
    const TuneKey k = tune_bucket(in_type, out_type, n_stations, n_channels, n_times);
    key[0] = k.in;
    key[1] = k.out;
    key[2] = k.sb;
    key[3] = k.gran;
    key[4] = k.tb;
    key[5] = k.ub;
    return XC_OK;
}

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
    const TuneKey key = tune_bucket(in_type, out_type, n_stations, n_channels, n_times);
    tune_put(key, best_c);
    log_line("tuned %d stations x %d channels x %d samples (in %d, out %d): kernel %d, block %d, time_chunk %d, "
             "time_split %d, staging %d, product %d, tile %dx%d, %.4f ms",
             n_stations, n_channels, n_times, (int)in_type, (int)out_type, best_c.kernel, best_c.block,
             best_c.time_chunk, best_c.time_split, best_c.staging, best_c.product, best_c.tile_w, best_c.tile_h,
             best_t);
    if (cache_path) {
        FILE *f = fopen(cache_path, "a");
        if (f) {
            fprintf(f,
                    "{\"in\": %d, \"out\": %d, \"sb\": %d, \"gran\": %d, \"tb\": %d, \"ub\": %d, \"kernel\": %d, "
                    "\"block\": %d, \"time_chunk\": %d, \"time_split\": %d, \"staging\": %d, \"product\": %d, "
                    "\"tile_w\": %d, \"tile_h\": %d, \"ms\": %.6f, \"S\": %d, \"C\": %d, \"T\": %d}\n",
                    key.in, key.out, key.sb, key.gran, key.tb, key.ub, best_c.kernel, best_c.block,
                    best_c.time_chunk, best_c.time_split, best_c.staging, best_c.product, best_c.tile_w,
                    best_c.tile_h, best_t, n_stations, n_channels, n_times);
            fclose(f);
        }
    }
    return XC_OK;
}

int64_t xc_tune_cache_load(const char *cache_path) {
    if (!cache_path) return -1;
    FILE *f = fopen(cache_path, "r");
    if (!f) return -1;
    char line[1024];
    int64_t n = 0;
    while (fgets(line, sizeof line, f)) {
        TuneKey key;
        xc_config c;
        double ms;
        int S, C, T;
        if (sscanf(line,
                   " {\"in\": %d, \"out\": %d, \"sb\": %d, \"gran\": %d, \"tb\": %d, \"ub\": %d, \"kernel\": %d, "
                   "\"block\": %d, \"time_chunk\": %d, \"time_split\": %d, \"staging\": %d, \"product\": %d, "
                   "\"tile_w\": %d, \"tile_h\": %d, \"ms\": %lf, \"S\": %d, \"C\": %d, \"T\": %d",
                   &key.in, &key.out, &key.sb, &key.gran, &key.tb, &key.ub, &c.kernel, &c.block, &c.time_chunk,
                   &c.time_split, &c.staging, &c.product, &c.tile_w, &c.tile_h, &ms, &S, &C, &T) != 18)
            continue;
        // keep the entry only if it still resolves for the shape it was tuned on
        xc_config r;
        if (xc_resolve_config(&c, (xc_in_type)key.in, (xc_out_type)key.out, S, 2, C, T, &r) != XC_OK) continue;
        const TuneKey k2 = tune_bucket(key.in, key.out, S, C, T);
        if (!(k2 == key)) continue;
        tune_put(key, r);
        ++n;
    }
    fclose(f);
    log_line("tune cache %s: %lld entries loaded", cache_path, (long long)n);
    return n;
}

}  // extern "C"
