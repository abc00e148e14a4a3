// Host ingest: correlation of samples that live in host memory.
//
// The paper finds GPU correlators bound by the host-to-device link
// (Section 3.6: perf_max,global = AI_global x host bandwidth, with
// AI_global = S + 1 flops per byte of complex-float samples), shows that
// asynchronous copies overlapped with computation are essential (Section
// 4.4), that concurrent copies slow the kernel (Section 4.3), and turns the
// natural station-major layout into the time-major one the GPU reads
// coalesced, on host threads, overlapped with the GPU (Section 4.4, the
// memory-layout figure).
//
// Here the channels are split into groups; two device staging slots
// alternate, so that the copy of group g + 1 (on a copy stream of its own)
// runs while group g is transposed (station-major input only) and correlated
// on the caller's stream.  The transpose runs on the GPU: at HBM speed it
// costs a few per cent of the PCIe copy it follows, so it stays off the
// critical path without taking host cores.  Each group is correlated by the
// same kernels as device-resident input, into its slice of V (channels are
// independent, Section 2), so the results are identical to those of
// xc_correlate_config on the whole time-major block.
#include <algorithm>
#include <cstdint>

#include "common.h"
#include "transpose.h"

namespace xc {
xc_status resolve(const xc_config *cfg, xc_in_type in_type, xc_out_type out_type, int32_t S, int32_t P, int32_t C,
                  int32_t T, Plan *plan);
Job make_job(const void *samples, void *vis, int S, int C, int T, int block, int accumulate);
xc_status launch_plan(const Plan &plan, xc_in_type in_type, xc_out_type out_type, const Job &job,
                      hipStream_t stream);

namespace {

// Bytes of one station's dual-polarised sample at one time step.
int station_sample_bytes(xc_in_type t) {
    switch (t) {
    case XC_IN_CF32: return 16;
    case XC_IN_CI8: return 4;
    default: return 8;
    }
}

bool valid_in_type(int t) { return t >= XC_IN_CF32 && t <= XC_IN_CBF16; }

// Transpose of each channel's S x T matrix of station samples (E = 4, 8 or 16
// bytes) from x[c][s][t] to x[c][t][s].
hipError_t launch_transpose(const void *src, void *dst, xc_in_type in_type, int S, int C, int T,
                            hipStream_t stream) {
    const int64_t st = (int64_t)S * T;
    return launch_transpose_tiles(src, dst, station_sample_bytes(in_type), S, T, T, S, st, st, C, stream);
}

xc_status check_shape(xc_in_type in_type, int32_t S, int32_t P, int32_t C, int32_t T) {
    if (!valid_in_type(in_type)) return set_error(XC_ERR_INVALID_ARG, "invalid in_type %d", (int)in_type);
    if (P != 2) return set_error(XC_ERR_UNSUPPORTED, "n_pol = %d: only dual-polarised stations (2) are supported", P);
    if (S < 1 || C < 1 || T < 1)
        return set_error(XC_ERR_INVALID_ARG, "sizes must be >= 1 (S=%d C=%d T=%d)", S, C, T);
    return XC_OK;
}

}  // namespace
}  // namespace xc

using namespace xc;

struct xc_ingest {
    xc_in_type in_type;
    int32_t S, C, T, layout, group;
    size_t chan_bytes;          // bytes of one channel's samples
    void *raw[2] = {nullptr, nullptr};    // staging slots: the copied group
    void *tmaj[2] = {nullptr, nullptr};   // its time-major transpose (station-major input)
    hipStream_t copy_stream = nullptr;
    hipEvent_t copied[2] = {nullptr, nullptr};    // copy of the slot's group done
    hipEvent_t consumed[2] = {nullptr, nullptr};  // correlation of the slot's group done
    bool used[2] = {false, false};
};

static void ingest_free(xc_ingest *g) {
    for (int k = 0; k < 2; ++k) {
        if (g->used[k]) (void)hipEventSynchronize(g->consumed[k]);
    }
    if (g->copy_stream) (void)hipStreamSynchronize(g->copy_stream);
    for (int k = 0; k < 2; ++k) {
        if (g->raw[k]) (void)hipFree(g->raw[k]);
        if (g->tmaj[k]) (void)hipFree(g->tmaj[k]);
        if (g->copied[k]) (void)hipEventDestroy(g->copied[k]);
        if (g->consumed[k]) (void)hipEventDestroy(g->consumed[k]);
    }
    if (g->copy_stream) (void)hipStreamDestroy(g->copy_stream);
    delete g;
}

extern "C" {

xc_status xc_transpose_to_time_major(const void *src, void *dst, xc_in_type in_type, int32_t n_stations,
                                     int32_t n_pol, int32_t n_channels, int32_t n_times, void *stream) {
    xc_status st = check_shape(in_type, n_stations, n_pol, n_channels, n_times);
    if (st != XC_OK) return st;
    if (!src || !dst) return set_error(XC_ERR_INVALID_ARG, "null src or dst pointer");
    if (src == dst) return set_error(XC_ERR_INVALID_ARG, "the transpose is out of place (src == dst)");
    const size_t E = (size_t)station_sample_bytes(in_type);
    if (((uintptr_t)src % E) || ((uintptr_t)dst % E))
        return set_error(XC_ERR_INVALID_ARG, "src and dst must be aligned to the %zu-byte station sample", E);
    const hipError_t e = launch_transpose(src, dst, in_type, n_stations, n_channels, n_times,
                                          static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_error(e, "transpose launch");
    return XC_OK;
}

xc_status xc_ingest_create(xc_in_type in_type, int32_t n_stations, int32_t n_pol, int32_t n_channels,
                           int32_t n_times, int32_t layout, int32_t channels_per_group, xc_ingest **out) {
    if (!out) return set_error(XC_ERR_INVALID_ARG, "null output pointer");
    *out = nullptr;
    xc_status st = check_shape(in_type, n_stations, n_pol, n_channels, n_times);
    if (st != XC_OK) return st;
    if (layout != XC_LAYOUT_TIME_MAJOR && layout != XC_LAYOUT_STATION_MAJOR)
        return set_error(XC_ERR_INVALID_ARG, "invalid layout %d", layout);
    if (channels_per_group < 0) return set_error(XC_ERR_INVALID_ARG, "channels_per_group must be >= 0");
    const size_t chan = (size_t)n_times * n_stations * station_sample_bytes(in_type);
    int32_t grp = channels_per_group;
    // default: about 128 MiB per group.  Each copy has a fixed cost of some
    // tens of microseconds; with the correlation tens of times faster than the
    // link, few large groups beat a finer pipeline (measured: 8 MiB groups
    // lose about a quarter of the rate).
    if (grp == 0) grp = (int32_t)std::max<size_t>(1, ((size_t)128 << 20) / chan);
    grp = std::min(grp, n_channels);
    xc_ingest *g = new xc_ingest;
    g->in_type = in_type;
    g->S = n_stations;
    g->C = n_channels;
    g->T = n_times;
    g->layout = layout;
    g->group = grp;
    g->chan_bytes = chan;
    const size_t bytes = chan * (size_t)grp;
    hipError_t e = hipStreamCreateWithFlags(&g->copy_stream, hipStreamNonBlocking);
    for (int k = 0; k < 2 && e == hipSuccess; ++k) {
        e = hipMalloc(&g->raw[k], bytes);
        if (e == hipSuccess && layout == XC_LAYOUT_STATION_MAJOR) e = hipMalloc(&g->tmaj[k], bytes);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&g->copied[k], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&g->consumed[k], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        ingest_free(g);
        return e == hipErrorOutOfMemory ? set_error(XC_ERR_OUT_OF_MEMORY, "staging buffers of %zu bytes", bytes)
                                        : hip_error(e, "ingest setup");
    }
    *out = g;
    return XC_OK;
}

xc_status xc_ingest_info(const xc_ingest *g, int32_t *channels_per_group, int64_t *device_bytes) {
    if (!g) return set_error(XC_ERR_INVALID_ARG, "null ingest");
    if (channels_per_group) *channels_per_group = g->group;
    if (device_bytes)
        *device_bytes = (int64_t)(g->chan_bytes * g->group * (g->layout == XC_LAYOUT_STATION_MAJOR ? 4 : 2));
    return XC_OK;
}

xc_status xc_ingest_run(xc_ingest *g, const xc_config *cfg, const void *host_samples, void *vis,
                        xc_out_type out_type, int32_t accumulate, int32_t overlap, void *stream) {
    if (!g) return set_error(XC_ERR_INVALID_ARG, "null ingest");
    if (!host_samples || !vis) return set_error(XC_ERR_INVALID_ARG, "null samples or vis pointer");
    if ((uintptr_t)vis & 15u) return set_error(XC_ERR_INVALID_ARG, "vis must be 16-byte aligned");
    if (accumulate != 0 && accumulate != 1) return set_error(XC_ERR_INVALID_ARG, "accumulate must be 0 or 1");
    if (overlap != 0 && overlap != 1) return set_error(XC_ERR_INVALID_ARG, "overlap must be 0 or 1");
    // one configuration for every group (a smaller last group resolves the same way)
    Plan plan;
    xc_status st = resolve(cfg, g->in_type, out_type, g->S, 2, g->group, g->T, &plan);
    if (st != XC_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // station-major complex float32 on a kernel whose sample loads corner-turn
    // (64-station matrix cores, vector ALU) is correlated as staged, without
    // the transpose
    const bool direct = g->layout == XC_LAYOUT_STATION_MAJOR && g->in_type == XC_IN_CF32 &&
                        (plan.kernel == XC_KERNEL_VALU || (plan.kernel == XC_KERNEL_MFMA && plan.block == 64));
    const size_t vis_chan = (size_t)g->S * (g->S + 1) / 2 * 4 * 8;   // bytes of one channel's V
    const uint8_t *host = static_cast<const uint8_t *>(host_samples);
    const int ngroups = (g->C + g->group - 1) / g->group;
    hipError_t e = hipSuccess;
    for (int k = 0; k < ngroups && e == hipSuccess; ++k) {
        const int slot = k & 1;
        const int c0 = k * g->group;
        const int cg = std::min(g->group, g->C - c0);
        hipStream_t cs = overlap ? g->copy_stream : s;
        // the slot is free once the correlation of its previous group is done
        if (g->used[slot]) e = hipStreamWaitEvent(cs, g->consumed[slot], 0);
        if (e == hipSuccess)
            e = hipMemcpyAsync(g->raw[slot], host + (size_t)c0 * g->chan_bytes, (size_t)cg * g->chan_bytes,
                               hipMemcpyHostToDevice, cs);
        if (e == hipSuccess && overlap) {
            e = hipEventRecord(g->copied[slot], cs);
            if (e == hipSuccess) e = hipStreamWaitEvent(s, g->copied[slot], 0);
        }
        const void *src = g->raw[slot];
        if (e == hipSuccess && g->layout == XC_LAYOUT_STATION_MAJOR && !direct) {
            e = launch_transpose(g->raw[slot], g->tmaj[slot], g->in_type, g->S, cg, g->T, s);
            src = g->tmaj[slot];
        }
        if (e != hipSuccess) break;
        Job job = make_job(src, static_cast<uint8_t *>(vis) + (size_t)c0 * vis_chan, g->S, cg, g->T, plan.block,
                           accumulate);
        if (direct) job.sstride = g->T;
        st = launch_plan(plan, g->in_type, out_type, job, s);
        if (st != XC_OK) return st;
        e = hipEventRecord(g->consumed[slot], s);
        if (e == hipSuccess) g->used[slot] = true;
    }
    if (e != hipSuccess) return hip_error(e, "ingest enqueue");
    return XC_OK;
}

void xc_ingest_destroy(xc_ingest *g) {
    if (g) ingest_free(g);
}

}  // extern "C"
