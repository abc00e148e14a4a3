// C ABI: argument validation, configuration resolution, dispatch, cost model.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

#include "common.h"
#include "log.h"

namespace xc {

namespace {
thread_local std::string g_last_error;
}

xc_status set_error(xc_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

namespace {
std::mutex g_log_mu;
FILE *log_file() {
    static FILE *f = [] {
        const char *v = getenv("XC_LOG");
        if (!v || !*v || strcmp(v, "0") == 0) return (FILE *)nullptr;
        if (strcmp(v, "1") == 0 || strcmp(v, "stderr") == 0) return stderr;
        return fopen(v, "a");
    }();
    return f;
}
}  // namespace

void log_line(const char *fmt, ...) {
    FILE *f = log_file();
    if (!f) return;
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    std::lock_guard<std::mutex> lk(g_log_mu);
    fprintf(f, "[xengine] %s\n", buf);
    fflush(f);
}

xc_status hip_error(hipError_t err, const char *what) {
    return set_error(XC_ERR_HIP, "%s: %s (%d)", what, hipGetErrorString(err), (int)err);
}

int device_cu_count() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 256;
    return n;
}

static bool valid_in(int t) { return t >= XC_IN_CF32 && t <= XC_IN_CBF16; }
static bool valid_out(int t) { return t == XC_OUT_CF32 || t == XC_OUT_CI32; }

// Time steps per LDS stage of the MFMA kernels (fixed per variant).
static int mfma_chunk(xc_in_type t, int block) {
    switch (t) {
    case XC_IN_CI8: return 64;
    case XC_IN_CF16:
    case XC_IN_CBF16: return 32;
    default: return 16;
    }
}

// Tuned configurations chosen by xc_autotune for a shape (process-wide).
struct TuneEntry {
    TuneKey key;
    xc_config cfg;
};
static std::mutex g_tune_mu;
static TuneEntry *g_tune = nullptr;
static int g_tune_n = 0, g_tune_cap = 0;

static int ceil_log2(int64_t v) {
    int k = 0;
    while (((int64_t)1 << k) < v) ++k;
    return k;
}

TuneKey tune_bucket(int in_type, int out_type, int S, int C, int T) {
    const int gran = in_type == XC_IN_CI8 ? 4 : (in_type == XC_IN_CF32 ? 1 : 2);
    const int64_t nb = (S + 63) / 64;
    const int64_t units = (int64_t)C * (nb * (nb + 1) / 2);
    // station classes: 32-station blocks, and arrays of at most 16 stations
    // apart (class 0), which have a kernel of their own
    const int sclass = S <= 16 ? 0 : (S + 31) / 32;
    return TuneKey{in_type, out_type, sclass, S % gran == 0 ? 1 : 0, ceil_log2(T), std::min(ceil_log2(units), 12)};
}

void tune_put(const TuneKey &k, const xc_config &cfg) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (int i = 0; i < g_tune_n; ++i)
        if (g_tune[i].key == k) {
            g_tune[i].cfg = cfg;
            return;
        }
    if (g_tune_n == g_tune_cap) {
        int cap = g_tune_cap ? 2 * g_tune_cap : 16;
        TuneEntry *n = static_cast<TuneEntry *>(realloc(g_tune, sizeof(TuneEntry) * cap));
        if (!n) return;
        g_tune = n;
        g_tune_cap = cap;
    }
    g_tune[g_tune_n++] = TuneEntry{k, cfg};
}

bool tune_get(const TuneKey &k, xc_config *cfg) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (int i = 0; i < g_tune_n; ++i)
        if (g_tune[i].key == k) {
            *cfg = g_tune[i].cfg;
            return true;
        }
    return false;
}

xc_status resolve(const xc_config *cfg_in, xc_in_type in_type, xc_out_type out_type, int32_t S, int32_t P,
                  int32_t C, int32_t T, Plan *plan) {
    if (!valid_in(in_type)) return set_error(XC_ERR_INVALID_ARG, "invalid in_type %d", (int)in_type);
    if (!valid_out(out_type)) return set_error(XC_ERR_INVALID_ARG, "invalid out_type %d", (int)out_type);
    if (P != 2) return set_error(XC_ERR_UNSUPPORTED, "n_pol = %d: only dual-polarised stations (2) are supported", P);
    if (S < 1 || C < 1 || T < 1)
        return set_error(XC_ERR_INVALID_ARG, "sizes must be >= 1 (S=%d C=%d T=%d)", S, C, T);
    if (S > 32768) return set_error(XC_ERR_UNSUPPORTED, "n_stations = %d exceeds 32768", S);
    if (out_type == XC_OUT_CI32 && in_type != XC_IN_CI8)
        return set_error(XC_ERR_INVALID_ARG, "XC_OUT_CI32 requires XC_IN_CI8 samples");
    if (out_type == XC_OUT_CI32 && T > XC_CI32_MAX_TIMES)
        return set_error(XC_ERR_OVERFLOW_RISK, "n_times = %d > %d: int32 visibilities could overflow", T,
                         XC_CI32_MAX_TIMES);

    xc_config cfg = {0, 0, 0, 0, 0, 0, 0, 0};
    if (cfg_in) cfg = *cfg_in;
    if (cfg.kernel == XC_KERNEL_AUTO && !cfg_in) {
        xc_config tuned;
        if (tune_get(tune_bucket((int)in_type, (int)out_type, S, C, T), &tuned)) cfg = tuned;
    }
    int kernel = cfg.kernel;
    // complex float32 on at most 16 stations: the one-channel kernel (8
    // stations x 16 channels x 256 samples: 6.2 us per launch against 21-25 us
    // for the block-pair kernels, whose chunk loop waits on its loads; 16
    // stations x 256 channels x 768 samples: 27 against 49-69 us)
    const bool small_auto = kernel == XC_KERNEL_AUTO && in_type == XC_IN_CF32 && S <= 16 && !cfg.block &&
                            !cfg.time_chunk && !cfg.time_split && !cfg.tile_w && !cfg.tile_h;
    if (small_auto) kernel = XC_KERNEL_VALU;
    if (kernel == XC_KERNEL_AUTO) kernel = XC_KERNEL_MFMA;
    if (kernel != XC_KERNEL_VALU && kernel != XC_KERNEL_MFMA)
        return set_error(XC_ERR_INVALID_ARG, "invalid kernel %d", cfg.kernel);
    if (cfg.staging < XC_STAGING_AUTO || cfg.staging > XC_STAGING_LDS)
        return set_error(XC_ERR_INVALID_ARG, "invalid staging %d", cfg.staging);
    if (cfg.product < XC_PRODUCT_AUTO || cfg.product > XC_PRODUCT_THREE)
        return set_error(XC_ERR_INVALID_ARG, "invalid product %d", cfg.product);
    Plan p;
    p.product = XC_PRODUCT_FOUR;
    p.kernel = kernel;
    p.tile_w = p.tile_h = 0;
    if (kernel == XC_KERNEL_VALU) {
        if (in_type != XC_IN_CF32)
            return set_error(XC_ERR_UNSUPPORTED, "the vector-ALU kernel takes complex-float32 samples only");
        p.block = cfg.block ? cfg.block : (small_auto ? 16 : 32);
        p.staging = cfg.staging ? cfg.staging : XC_STAGING_REGISTERS;
        if (p.staging != XC_STAGING_REGISTERS)
            return set_error(XC_ERR_INVALID_ARG, "the vector-ALU kernels stage through registers only");
        if (p.block == 16) {
            // one workgroup per channel, all baselines; its chunk (128 time
            // steps) and time groups (up to 32) are fixed
            if (S > 16) return set_error(XC_ERR_INVALID_ARG, "VALU block 16 takes at most 16 stations (got %d)", S);
            if (cfg.tile_w || cfg.tile_h)
                return set_error(XC_ERR_INVALID_ARG, "VALU block 16 has no register tiles (tile_w, tile_h must be 0)");
            if (cfg.time_chunk && cfg.time_chunk != 128)
                return set_error(XC_ERR_INVALID_ARG, "VALU block 16 stages chunks of 128 time steps");
            if (cfg.time_split > 1)
                return set_error(XC_ERR_INVALID_ARG, "VALU block 16 chooses its own time groups (time_split 0 or 1)");
            p.time_chunk = 128;
            p.time_split = 1;
        } else {
            p.time_chunk = cfg.time_chunk ? cfg.time_chunk : 32;
            p.time_split = cfg.time_split ? cfg.time_split : 4;
            // default 4 x 2 tiles, chunks of 32 time steps, four time groups: the
            // fastest measured configuration on 64 stations (74.7 TFLOP/s against
            // 73.1 for 2 x 2 tiles and 53.0 for 4 x 4) and within 1 % of the
            // fastest on 256 stations (85.1 against 85.4)
            p.tile_w = cfg.tile_w ? cfg.tile_w : 4;
            p.tile_h = cfg.tile_h ? cfg.tile_h : 2;
            if (p.block != 32) return set_error(XC_ERR_INVALID_ARG, "VALU block must be 32 or 16 (got %d)", p.block);
            if (!valu_available(p.tile_w, p.tile_h, p.time_chunk, p.time_split))
                return set_error(XC_ERR_INVALID_ARG,
                                 "VALU (tile %d x %d, time_chunk %d, time_split %d) not available", p.tile_w,
                                 p.tile_h, p.time_chunk, p.time_split);
        }
    } else {
        // complex-float32 on few stations: 64-station blocks would leave most
        // of their tiles empty (measured: 8, 24 and 40 stations run 15-20 %
        // faster on 32-station blocks; 64 stations twice as fast on 64)
        if (cfg.tile_w || cfg.tile_h)
            return set_error(XC_ERR_INVALID_ARG, "register tiles are a vector-ALU setting (tile_w, tile_h must be 0)");
        p.block = cfg.block ? cfg.block : (in_type == XC_IN_CF32 && S <= 48 ? 32 : 64);
        if (p.block != 32 && p.block != 64)
            return set_error(XC_ERR_INVALID_ARG, "MFMA block must be 32 or 64 (got %d)", p.block);
        // complex-float32 on 64-station blocks uses the 16x16 tile kernel, which
        // copies straight into LDS and can split time over two wave groups;
        // int8 and 16-bit samples on 64-station blocks take either staging
        // (AUTO: straight into LDS); the rest stage through registers
        const bool f16tile = in_type == XC_IN_CF32 && p.block == 64;
        const bool either = in_type != XC_IN_CF32 && p.block == 64;
        const bool lds_ok = f16tile || either;
        p.staging = cfg.staging ? cfg.staging : (lds_ok ? XC_STAGING_LDS : XC_STAGING_REGISTERS);
        if (p.staging == XC_STAGING_LDS && !lds_ok)
            return set_error(XC_ERR_INVALID_ARG, "this configuration stages through registers only");
        if (p.staging == XC_STAGING_REGISTERS && f16tile)
            return set_error(XC_ERR_INVALID_ARG,
                             "complex-float32 on 64-station blocks copies straight into LDS only");
        if (f16tile) p.product = cfg.product ? cfg.product : kDefaultProductF32;
        p.time_split = cfg.time_split ? cfg.time_split : (f16tile && S <= 64 ? 2 : 1);
        if (!(p.time_split == 1 || (f16tile && p.time_split == 2)))
            return set_error(XC_ERR_INVALID_ARG,
                             "MFMA time_split must be 1 (or 2 for complex-float32 on 64-station blocks)");
        const int chunk = f16tile ? (p.time_split == 2 ? 32 : 16) : mfma_chunk(in_type, p.block);
        p.time_chunk = cfg.time_chunk ? cfg.time_chunk : chunk;
        if (p.time_chunk != chunk)
            return set_error(XC_ERR_INVALID_ARG, "MFMA time_chunk for this configuration must be %d", chunk);
    }
    if (cfg.product == XC_PRODUCT_THREE && p.product != XC_PRODUCT_THREE)
        return set_error(XC_ERR_INVALID_ARG,
                         "the three-product form is available for complex-float32 on 64-station MFMA blocks only");
    const int64_t nb = (S + p.block - 1) / p.block;
    const int64_t nwork = (int64_t)C * (nb * (nb + 1) / 2);
    if (nwork > (int64_t)1 << 30)
        return set_error(XC_ERR_UNSUPPORTED, "too many work units (%lld)", (long long)nwork);
    *plan = p;
    return XC_OK;
}

static int in_bytes(xc_in_type t) {
    switch (t) {
    case XC_IN_CF32: return 8;
    case XC_IN_CI8: return 2;
    default: return 4;
    }
}

static bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// Pieces an integration of T steps is split into when n_split are asked for:
// pieces of ceil(T / n_split) steps, none empty.
static int32_t split_pieces(int32_t T, int32_t n_split) {
    const int32_t k = std::min(n_split, T);
    const int32_t len = (T + k - 1) / k;
    return (T + len - 1) / len;
}

// vis[e] (+)= sum over pieces k = 0 .. K-1, in that order, of part[k][e]: the
// time reduction of an integration split over workgroups, in a fixed order.
template <typename E>
__global__ void add_pieces(const E *__restrict__ part, E *__restrict__ vis, int64_t n, int K, int accumulate) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        E a = accumulate ? vis[e] : E{};
        for (int k = 0; k < K; ++k) {
            const E v = part[(int64_t)k * n + e];
            a.x += v.x;
            a.y += v.y;
        }
        vis[e] = a;
    }
}

// -- optional scan of int8 input for -128 (XC_CHECK=1) --
__global__ void scan_m128(const int8_t *x, size_t n, int *flag) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride)
        if (x[i] == -128) {
            *flag = 1;
            return;
        }
}
__global__ void zero_int(int *p) { *p = 0; }

static xc_status check_int8(const void *samples, size_t n, hipStream_t stream) {
    int *flag = nullptr;
    hipError_t e = hipMalloc(&flag, sizeof(int));
    if (e != hipSuccess) return hip_error(e, "hipMalloc(check flag)");
    hipLaunchKernelGGL(zero_int, dim3(1), dim3(1), 0, stream, flag);
    hipLaunchKernelGGL(scan_m128, dim3(1024), dim3(256), 0, stream, static_cast<const int8_t *>(samples), n, flag);
    int h = 0;
    e = hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    (void)hipFree(flag);
    if (e != hipSuccess) return hip_error(e, "XC_CHECK scan");
    if (h) return set_error(XC_ERR_INVALID_ARG, "XC_CHECK: int8 samples contain -128 (domain is [-127, 127])");
    return XC_OK;
}

static bool check_env() {
    const char *v = getenv("XC_CHECK");
    return v && v[0] == '1';
}

Job make_job(const void *samples, void *vis, int S, int C, int T, int block, int accumulate) {
    Job j;
    j.x = samples;
    j.vis = vis;
    j.S = S;
    j.C = C;
    j.T = T;
    j.nb = (S + block - 1) / block;
    j.npairs = j.nb * (j.nb + 1) / 2;
    j.accumulate = accumulate ? 1 : 0;
    j.tblk = T;
    j.bstride = 0;
    j.slot0 = 0;
    j.nring = 1 << 30;
    j.cstride = (int64_t)T * S;
    j.tsplit = 1;
    j.tpiece = T;
    j.xpiece = 0;
    j.vpiece = 0;
    j.sstride = 0;
    return j;
}

xc_status launch_plan(const Plan &plan, xc_in_type in_type, xc_out_type out_type, const Job &job,
                      hipStream_t stream) {
    hipError_t e;
    if (plan.kernel == XC_KERNEL_VALU) e = launch_valu(plan, job, stream);
    else if (in_type == XC_IN_CF32 && plan.block == 64) e = launch_mfma16(plan, job, stream);
    else if (plan_is_dma(plan, in_type)) e = launch_mfma_dma(in_type, out_type, job, stream);
    else e = launch_mfma(plan, in_type, out_type, job, stream);
    if (e != hipSuccess) return hip_error(e, "kernel launch");
    return XC_OK;
}

}  // namespace xc

using namespace xc;

extern "C" {

int64_t xc_n_baselines(int32_t n_stations) {
    if (n_stations < 0) return -1;
    return (int64_t)n_stations * (n_stations + 1) / 2;
}

int64_t xc_baseline_index(int32_t i, int32_t j) {
    if (i < 0 || j < 0 || i > j) return -1;
    return (int64_t)j * (j + 1) / 2 + i;
}

int64_t xc_vis_elems(int32_t n_stations, int32_t n_pol, int32_t n_channels) {
    if (n_stations < 0 || n_pol < 0 || n_channels < 0) return -1;
    return (int64_t)n_channels * xc_n_baselines(n_stations) * n_pol * n_pol;
}

int64_t xc_sample_bytes(xc_in_type in_type, int32_t n_stations, int32_t n_pol, int32_t n_channels,
                        int32_t n_times) {
    if (!valid_in(in_type) || n_stations < 0 || n_pol < 0 || n_channels < 0 || n_times < 0) return -1;
    return (int64_t)n_channels * n_times * n_stations * n_pol * in_bytes(in_type);
}

int64_t xc_vis_bytes(xc_out_type out_type, int32_t n_stations, int32_t n_pol, int32_t n_channels) {
    if (!valid_out(out_type)) return -1;
    const int64_t n = xc_vis_elems(n_stations, n_pol, n_channels);
    return n < 0 ? -1 : n * 8;
}

xc_status xc_resolve_config(const xc_config *cfg, xc_in_type in_type, xc_out_type out_type, int32_t n_stations,
                            int32_t n_pol, int32_t n_channels, int32_t n_times, xc_config *resolved) {
    Plan p;
    xc_status st = resolve(cfg, in_type, out_type, n_stations, n_pol, n_channels, n_times, &p);
    if (st != XC_OK) return st;
    if (resolved) {
        resolved->kernel = p.kernel;
        resolved->block = p.block;
        resolved->time_chunk = p.time_chunk;
        resolved->time_split = p.time_split;
        resolved->staging = p.staging;
        resolved->product = p.product;
        resolved->tile_w = p.tile_w;
        resolved->tile_h = p.tile_h;
    }
    return XC_OK;
}

xc_status xc_correlate_config(const xc_config *cfg, const void *samples, xc_in_type in_type, int32_t n_stations,
                              int32_t n_pol, int32_t n_channels, int32_t n_times, void *vis,
                              xc_out_type out_type, int32_t accumulate, void *stream) {
    Plan plan;
    xc_status st = resolve(cfg, in_type, out_type, n_stations, n_pol, n_channels, n_times, &plan);
    if (st != XC_OK) return st;
    if (!samples || !vis) return set_error(XC_ERR_INVALID_ARG, "null samples or vis pointer");
    if (!aligned16(samples) || !aligned16(vis))
        return set_error(XC_ERR_INVALID_ARG, "samples and vis must be 16-byte aligned");
    if (accumulate != 0 && accumulate != 1) return set_error(XC_ERR_INVALID_ARG, "accumulate must be 0 or 1");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (in_type == XC_IN_CI8 && check_env()) {
        st = check_int8(samples, (size_t)xc_sample_bytes(in_type, n_stations, n_pol, n_channels, n_times), s);
        if (st != XC_OK) return st;
    }
    const Job job = make_job(samples, vis, n_stations, n_channels, n_times, plan.block, accumulate);
    return launch_plan(plan, in_type, out_type, job, s);
}

int64_t xc_correlate_split_bytes(int32_t n_stations, int32_t n_pol, int32_t n_channels, int32_t n_times,
                                 int32_t n_split) {
    if (n_stations < 1 || n_pol != 2 || n_channels < 1 || n_times < 1 || n_split < 1) return -1;
    const int32_t K = split_pieces(n_times, n_split);
    return (int64_t)K * xc_vis_elems(n_stations, n_pol, n_channels) * 8;
}

// The integration split over workgroups once the workspace is known: the K
// pieces' partial sums into `work` (every element written, so it need not be
// cleared), then vis (+)= their sum in the fixed order k = 0 .. K-1.
static xc_status split_run(const Plan &plan, const void *samples, xc_in_type in_type, int32_t S, int32_t C,
                           int32_t T, void *vis, xc_out_type out_type, int32_t accumulate, int32_t K, void *work,
                           hipStream_t s) {
    const int64_t elems = xc_vis_elems(S, 2, C);
    Job job = make_job(samples, work, S, C, T, plan.block, 0);
    job.tsplit = K;
    job.tpiece = (T + K - 1) / K;
    job.xpiece = (int64_t)job.tpiece * S * 2 * in_bytes(in_type);
    job.vpiece = elems * 8;
    if ((int64_t)job.C * job.npairs * K > ((int64_t)1 << 30))
        return set_error(XC_ERR_UNSUPPORTED, "too many work units");
    xc_status st = launch_plan(plan, in_type, out_type, job, s);
    if (st != XC_OK) return st;
    const int blocks = (int)std::min<int64_t>((elems + 255) / 256, 65536);
    if (out_type == XC_OUT_CI32)
        hipLaunchKernelGGL(add_pieces<int2>, dim3(blocks), dim3(256), 0, s, static_cast<const int2 *>(work),
                           static_cast<int2 *>(vis), elems, K, accumulate);
    else
        hipLaunchKernelGGL(add_pieces<float2>, dim3(blocks), dim3(256), 0, s, static_cast<const float2 *>(work),
                           static_cast<float2 *>(vis), elems, K, accumulate);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "piece-sum launch");
    return XC_OK;
}

// Scratch of xc_correlate_split_static: one array per device, kept until the
// process ends.  Host code reaches it only through the device address that
// hipGetSymbolAddress returns for the current device (the array's name in host
// code is not a device address).
static __device__ __align__(256) uint8_t scratch[XC_SPLIT_STATIC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
static void *g_scratch_dev[kMaxDevices];

static xc_status static_scratch(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_error(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return set_error(XC_ERR_UNSUPPORTED, "device %d: too many devices", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return XC_OK;
}

xc_status xc_correlate_split(const xc_config *cfg, const void *samples, xc_in_type in_type, int32_t n_stations,
                             int32_t n_pol, int32_t n_channels, int32_t n_times, void *vis, xc_out_type out_type,
                             int32_t accumulate, int32_t n_split, void *work, int64_t work_bytes, void *stream) {
    if (n_split < 1) return set_error(XC_ERR_INVALID_ARG, "n_split must be >= 1");
    const int32_t K = n_times >= 1 ? split_pieces(n_times, n_split) : 1;
    if (K == 1)
        return xc_correlate_config(cfg, samples, in_type, n_stations, n_pol, n_channels, n_times, vis, out_type,
                                   accumulate, stream);
    Plan plan;
    xc_status st = resolve(cfg, in_type, out_type, n_stations, n_pol, n_channels, n_times, &plan);
    if (st != XC_OK) return st;
    if (!samples || !vis || !work) return set_error(XC_ERR_INVALID_ARG, "null samples, vis or work pointer");
    if (!aligned16(samples) || !aligned16(vis) || !aligned16(work))
        return set_error(XC_ERR_INVALID_ARG, "samples, vis and work must be 16-byte aligned");
    if (accumulate != 0 && accumulate != 1) return set_error(XC_ERR_INVALID_ARG, "accumulate must be 0 or 1");
    const int64_t elems = xc_vis_elems(n_stations, n_pol, n_channels);
    if (work_bytes < (int64_t)K * elems * 8)
        return set_error(XC_ERR_INVALID_ARG, "work holds %lld bytes, %lld needed", (long long)work_bytes,
                         (long long)K * elems * 8);
    return split_run(plan, samples, in_type, n_stations, n_channels, n_times, vis, out_type, accumulate, K, work,
                     static_cast<hipStream_t>(stream));
}

xc_status xc_correlate_split_static(const xc_config *cfg, const void *samples, xc_in_type in_type,
                                    int32_t n_stations, int32_t n_pol, int32_t n_channels, int32_t n_times, void *vis,
                                    xc_out_type out_type, int32_t accumulate, int32_t n_split, void *stream) {
    if (n_split < 1) return set_error(XC_ERR_INVALID_ARG, "n_split must be >= 1");
    Plan plan;
    xc_status st = resolve(cfg, in_type, out_type, n_stations, n_pol, n_channels, n_times, &plan);
    if (st != XC_OK) return st;
    if (!samples || !vis) return set_error(XC_ERR_INVALID_ARG, "null samples or vis pointer");
    if (!aligned16(samples) || !aligned16(vis))
        return set_error(XC_ERR_INVALID_ARG, "samples and vis must be 16-byte aligned");
    if (accumulate != 0 && accumulate != 1) return set_error(XC_ERR_INVALID_ARG, "accumulate must be 0 or 1");
    const int32_t K = split_pieces(n_times, n_split);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (K == 1) {
        const Job job = make_job(samples, vis, n_stations, n_channels, n_times, plan.block, accumulate);
        return launch_plan(plan, in_type, out_type, job, s);
    }
    const int64_t need = (int64_t)K * xc_vis_elems(n_stations, n_pol, n_channels) * 8;
    if (need > (int64_t)XC_SPLIT_STATIC_SCRATCH_BYTES)
        return set_error(XC_ERR_UNSUPPORTED, "%d pieces of %lld visibilities need %lld bytes of scratch, more than %lld",
                         K, (long long)xc_vis_elems(n_stations, n_pol, n_channels), (long long)need,
                         (long long)XC_SPLIT_STATIC_SCRATCH_BYTES);
    void *work = nullptr;
    st = static_scratch(&work);
    if (st != XC_OK) return st;
    return split_run(plan, samples, in_type, n_stations, n_channels, n_times, vis, out_type, accumulate, K, work, s);
}

xc_status xc_correlate_station_major(const xc_config *cfg, const void *samples, xc_in_type in_type,
                                     int32_t n_stations, int32_t n_pol, int32_t n_channels, int32_t n_times,
                                     void *vis, xc_out_type out_type, int32_t accumulate, void *stream) {
    // the kernels whose sample loads take either layout: the 64-station
    // matrix-core kernels that copy straight into LDS (complex float32 16 x 16
    // tiles; int8 and 16-bit samples in 4-byte copies) and the vector-ALU
    // kernels (complex float32, including the one-channel kernel)
    xc_config c = cfg ? *cfg : xc_config{};
    if (c.kernel == XC_KERNEL_AUTO) {
        // as for time-major input: the one-channel kernel for complex float32
        // on at most 16 stations, otherwise the 64-station matrix-core kernel
        const bool small = in_type == XC_IN_CF32 && n_stations <= 16 && !c.block && !c.time_chunk &&
                           !c.time_split && !c.tile_w && !c.tile_h;
        c.kernel = small ? XC_KERNEL_VALU : XC_KERNEL_MFMA;
        if (small) c.block = 16;
    }
    if (c.kernel == XC_KERNEL_MFMA && c.block != 0 && c.block != 64)
        return set_error(XC_ERR_UNSUPPORTED, "station-major input: the matrix-core kernel on 64-station blocks only");
    if (c.kernel == XC_KERNEL_MFMA) c.block = 64;
    if (in_type != XC_IN_CF32 && c.kernel == XC_KERNEL_MFMA) {
        if (c.staging == XC_STAGING_REGISTERS)
            return set_error(XC_ERR_UNSUPPORTED, "station-major int8 / 16-bit input is copied straight into LDS");
        c.staging = XC_STAGING_LDS;
    }
    Plan plan;
    xc_status st = resolve(&c, in_type, out_type, n_stations, n_pol, n_channels, n_times, &plan);
    if (st != XC_OK) return st;
    if (!(plan.kernel == XC_KERNEL_VALU || (plan.kernel == XC_KERNEL_MFMA && plan.block == 64)))
        return set_error(XC_ERR_UNSUPPORTED, "station-major input: the matrix-core kernel on 64-station blocks only");
    if (!samples || !vis) return set_error(XC_ERR_INVALID_ARG, "null samples or vis pointer");
    if (!aligned16(samples) || !aligned16(vis))
        return set_error(XC_ERR_INVALID_ARG, "samples and vis must be 16-byte aligned");
    if (accumulate != 0 && accumulate != 1) return set_error(XC_ERR_INVALID_ARG, "accumulate must be 0 or 1");
    Job job = make_job(samples, vis, n_stations, n_channels, n_times, plan.block, accumulate);
    job.sstride = n_times;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (in_type != XC_IN_CF32) {
        const hipError_t e = launch_mfma_dma_station_major(in_type, out_type, job, s);
        if (e != hipSuccess) return hip_error(e, "kernel launch");
        return XC_OK;
    }
    return launch_plan(plan, in_type, out_type, job, s);
}

xc_status xc_correlate(const void *samples, xc_in_type in_type, int32_t n_stations, int32_t n_pol,
                       int32_t n_channels, int32_t n_times, void *vis, xc_out_type out_type, int32_t accumulate,
                       void *stream) {
    return xc_correlate_config(nullptr, samples, in_type, n_stations, n_pol, n_channels, n_times, vis, out_type,
                               accumulate, stream);
}

xc_status xc_tile_cost(int32_t w, int32_t h, int64_t *flops, int64_t *bytes, int64_t *min_registers) {
    if (w < 1 || h < 1 || !flops || !bytes || !min_registers)
        return set_error(XC_ERR_INVALID_ARG, "tile sizes must be >= 1 and outputs non-null");
    // Table 1: a w x h tile correlates w stations with h stations, 4 polarisation
    // products of 8 flops each per station pair and time step, from w + h
    // dual-polarised complex-float samples of 16 bytes.  Registers: 8 floats of
    // accumulators per station pair, plus the samples of one side (4 floats
    // each) and one sample of the other side.
    *flops = 32LL * w * h;
    *bytes = 16LL * (w + h);
    *min_registers = 4LL * (1 + (w < h ? w : h)) + 8LL * w * h;
    return XC_OK;
}

double xc_perf_max(double perf_peak, double arithmetic_intensity, double bandwidth) {
    const double mem = arithmetic_intensity * bandwidth;
    return perf_peak < mem ? perf_peak : mem;
}

double xc_ai_global(int32_t n_stations) {
    if (n_stations < 1) return NAN;
    // 32 flops x S(S+1)/2 baselines over 16 bytes x S stations
    return 32.0 * ((double)n_stations * (n_stations + 1) / 2.0) / (16.0 * n_stations);
}

double xc_flops(int32_t n_stations, int32_t n_channels, int32_t n_times) {
    return 32.0 * n_channels * (double)n_times * ((double)n_stations * (n_stations + 1) / 2.0);
}

const char *xc_status_string(xc_status status) {
    switch (status) {
    case XC_OK: return "XC_OK";
    case XC_ERR_INVALID_ARG: return "XC_ERR_INVALID_ARG";
    case XC_ERR_UNSUPPORTED: return "XC_ERR_UNSUPPORTED";
    case XC_ERR_OUT_OF_MEMORY: return "XC_ERR_OUT_OF_MEMORY";
    case XC_ERR_OVERFLOW_RISK: return "XC_ERR_OVERFLOW_RISK";
    case XC_ERR_ADMISSION: return "XC_ERR_ADMISSION";
    case XC_ERR_BACKPRESSURE: return "XC_ERR_BACKPRESSURE";
    case XC_ERR_HIP: return "XC_ERR_HIP";
    case XC_ERR_STATE: return "XC_ERR_STATE";
    }
    return "XC_ERR_UNKNOWN";
}

const char *xc_last_error(void) { return g_last_error.c_str(); }

const char *xc_version(void) { return "xengine 0.1 (gfx950)"; }

}  // extern "C"
